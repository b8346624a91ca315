"""Shared test plumbing: builds the same seeded inputs for the oracle and
the HIP path (each from its own tables) and compares results."""
from __future__ import annotations

import numpy as np
import torch

import workloads as W
from oracle import mesh as omesh
from oracle import solver as osolver


def strain_components(S, d):
    """(n, d, d) -> (NS, n) in the library's order xx, yy[, zz], xy[, yz, xz]."""
    if d == 3:
        idx = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]
    else:
        idx = [(0, 0), (1, 1), (0, 1)]
    return np.stack([S[:, a, b] for a, b in idx], 0)


def level_positions_from_coords(coords, level, level0):
    """coords (d, n) -> barycentres (n, d) in level0 cell units."""
    return (coords.T.astype(np.float64) + 0.5) / float(1 << (level - level0))


def fields_for(positions_by_level, level0, field_fn):
    """field_fn(pos) -> (rho, u, S) in level0 units; returns per-level dicts
    with S converted to level units."""
    rho, u, S = {}, {}, {}
    for L, pos in positions_by_level.items():
        r, uu, SS = field_fn(pos)
        rho[L], u[L], S[L] = r, uu, SS * 2.0 ** -(L - level0)
    return rho, u, S


def oracle_run(spec, tau0, field_fn, steps, u_in=None, poison=True, om=None, walls=None):
    om = om or omesh.build(spec)
    pos = {L: om.positions(L)[:om.lev(L).n_fluid] for L in range(om.level0, om.lmax + 1)}
    rho, u, S = fields_for(pos, om.level0, field_fn)
    sim = osolver.OracleSim(om, tau0, u_in=None if u_in is None else torch.tensor(u_in),
                            poison=poison, walls=walls)
    sim.init(rho, u, S)
    sim.step(steps)
    return sim


def gpu_sim(spec, precision, tau0, field_fn, u_in=None, f16_exp=None, plan=None):
    import paper_1601_06984_amd as M
    plan = plan or M.Plan.from_spec(spec)
    sim = M.Sim(plan, precision, tau0, u_in=u_in, f16_exp=f16_exp)
    dev = sim.device
    for k in range(plan.n_levels):
        L = plan.level0 + k
        nf = plan.info[k]["n_fluid"]
        coords = plan.export(k, "coords")[:, :nf]
        pos = level_positions_from_coords(coords, L, plan.level0)
        r, uu, SS = field_fn(pos)
        SS = SS * 2.0 ** -(L - plan.level0)
        sim.init(k, torch.tensor(r, device=dev), torch.tensor(np.ascontiguousarray(uu.T), device=dev),
                 torch.tensor(np.ascontiguousarray(strain_components(SS, plan.d)), device=dev))
    sim.fill_ghosts()
    return sim


def direction_perm(stencil, olat):
    import paper_1601_06984_amd as M
    c, _ = M.lattice(stencil)
    return [int(np.where((olat.c == c[i]).all(1))[0][0]) for i in range(len(c))]


def gpu_to_oracle(plan, om, k):
    """Index map: element g of the library's level k -> oracle index (the
    two layouts hold the same treeIDs; only the fluid order may differ)."""
    gt = plan.export(k, "treeid")
    ot = om.lev(om.level0 + k).tid
    order = np.argsort(ot)
    pos = np.searchsorted(ot[order], gt)
    g2o = order[np.minimum(pos, len(ot) - 1)]
    assert np.array_equal(ot[g2o], gt), "element sets differ"
    return g2o


def compare_post(sim, osim, fluid_only=False):
    """Max relative difference of post-collision pdfs over all levels."""
    perm = direction_perm(sim.plan.stencil, osim.lat)
    worst = 0.0
    for k in range(sim.plan.n_levels):
        L = sim.plan.level0 + k
        g = sim.get_pdf(k).cpu().numpy()
        g2o = gpu_to_oracle(sim.plan, osim.mesh, k)
        o = osim.post_collision(L).detach().numpy()[perm][:, g2o]
        n = sim.plan.info[k]["n_fluid"] if fluid_only else g.shape[1]
        rel = np.abs(g[:, :n] - o[:, :n]) / np.abs(o[:, :n])
        assert np.isfinite(o[:, :n]).all()
        worst = max(worst, float(rel.max()) if rel.size else 0.0)
    return worst


def tgv(n0, u0):
    return lambda pos: W.tgv_fields(pos, n0, u0)
