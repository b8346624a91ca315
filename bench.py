"""Benchmark of the multilevel lattice Boltzmann hot path on one MI355X.

One step = one coarse time step of the whole multilevel method (every
level's stream-collide with captures, both interpolation fills) over the
workload's mesh.  Throughput is reported in MLUPS with the paper's
workload weight: each fluid element of level L counts 2^(L-L0) updates per
coarse step.

The default workload is the largest single-GPU configuration: the
four-level D3Q19 sphere channel of 449 M elements with FP16-shifted pdf
storage and FP32 collision.  Prints ONE JSON line.  `roofline` is measured
live for the dominant kernel (the finest level's stream-collide) with HIP
events recorded on the stream the kernels run on, and priced with the
algorithmic bytes of the method (q pdfs read and written plus an int32
neighbour index per moving direction); the adjoint leg, an FP32 run of the
same mesh, the fixed-error precision study on the two-level Taylor-Green
box and `cpu_baseline` (the FP64 oracle, single-threaded, on a bounded
sample) follow.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "MLUPS & %HBM peak, fwd and adjoint step, FP32 vs FP16-shift at fixed error"
HBM_PEAK_GBS = 8000.0
INFINITY_CACHE_BYTES = 256 << 20
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16s": 2}


def algorithmic_bytes(q, prec):
    """What one fluid update must move: q pdfs read and q written at the
    storage width, plus an int32 pull index per moving direction."""
    return 2 * q * STORAGE_BYTES[prec] + 4 * (q - 1)


def algorithmic_bytes_adjoint(q, prec):
    """One reverse update: the forward pdfs re-read (q at the storage
    width), the pull indices, lambda read and written in the compute
    precision (FP32; FP64 in the F64 variant)."""
    lam = 8 if prec == "f64" else 4
    return q * STORAGE_BYTES[prec] + 4 * (q - 1) + 2 * q * lam


# HBM bytes per stream-collide launch (average over the level's launches,
# which alternate between the fluid range and fluid plus the inner ghosts),
# from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) of this bench
# on MI355X, each scaled by what the counter reads for a plain 1536 MiB
# device copy (fetch x 2.0, write x 1.0).  Summary and commands:
# profiles/stream_collide_sphere4_f16s.md.  The figures belong to the
# kernel sources they were measured on (KERNEL_SOURCES digest); with any
# other source the bench reports traffic as null.
PMC_TRAFFIC = {
    "sources_sha256_16": "fc12edafced1c302",
    "bytes_per_launch": {
        "sphere4/f16s/10": 19713010592,
        "sphere4/f16s/11": 7154536325,
        "sphere4/f16s/12": 7154536325,
        "sphere4/f16s/13": 7652108709,
    },
}
KERNEL_SOURCES = ("kernels.hpp", "launch.hpp", "common.hpp")


def calib_gather(torch, nbytes, m=1 << 22, reps=3):
    """Three gathers of m 2-byte values at seeded uniform random positions of
    a never-touched buffer of nbytes (torch.index_select, one kernel each,
    each with its own positions), and the distinct 64- and 128-byte lines
    each one touches, for reading FETCH_SIZE on partial-line requests."""
    import numpy as np
    n = nbytes // 2
    buf = torch.empty(n, dtype=torch.float16, device="cuda")
    rng = np.random.default_rng(1601)
    runs = []
    for _ in range(reps):
        idx = np.sort(rng.integers(0, n, size=m))
        runs.append({"values": m, "index_bytes": 8 * m, "out_bytes": 2 * m,
                     "distinct_64B_lines": int(np.unique(idx >> 5).size),
                     "distinct_128B_lines": int(np.unique(idx >> 6).size)})
        it = torch.from_numpy(idx).to("cuda")
        torch.index_select(buf, 0, it)
        torch.cuda.synchronize()
        del it
    del buf
    return {"buffer_bytes": nbytes, "runs": runs}


def kernel_sources_digest():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1601_06984_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name, precision, level):
    if kernel_sources_digest() != PMC_TRAFFIC["sources_sha256_16"]:
        return None
    return PMC_TRAFFIC["bytes_per_launch"].get(f"{workload_name}/{precision}/{level}")


def tgv_tau(n0, u0=0.02, re=100.0):
    # Re = u0 N0 / (2 pi nu) in coarse lattice units; nu = (tau - 1/2)/3
    return 0.5 + 3.0 * u0 * n0 / (2.0 * math.pi * re)


def workload(name):
    wl = _workload(name)
    wl["name"] = name
    return wl


def _workload(name):
    # a "_q27" suffix runs the same workload on the D3Q27 lattice; a "_bz"
    # suffix gives a sphere workload curved walls (the fraction at which the
    # sphere cuts each link into it, linear interpolated bounce-back); a
    # "_diff" suffix runs a Taylor-Green workload under diffusive scaling
    # between levels (four fine steps per coarse step, four GhostFromCoarser
    # layers, one tau on every level)
    if name.endswith("_diff"):
        wl = _workload(name[:-5])
        if not wl.get("tgv"):
            raise SystemExit("diffusive scaling runs the Taylor-Green workloads")
        wl["diffusive"] = True
        wl["desc"] += "; diffusive scaling between levels (four fine steps per coarse step)"
        return wl
    stencil = "D3Q19"
    if name.endswith("_q27"):
        stencil, name = "D3Q27", name[:-4]
    if name.endswith("_bz"):
        wl = _workload(name[:-3] + ("_q27" if stencil == "D3Q27" else ""))
        if wl.get("tgv"):
            raise SystemExit("curved walls need a sphere workload")
        wl["walls"] = True
        wl["desc"] += "; curved walls (linear interpolated bounce-back)"
        return wl
    if name == "tgv64":
        n0, u0 = 64, 0.02
        spec = W.refined_box_mesh(stencil, 6, 16, 48)
        desc = (f"{stencil} periodic Taylor-Green vortex, 64^3 coarse with the central "
                "32^3 coarse cells refined once (2 levels), u0=0.02, Re=100")
        return dict(spec=spec, tau0=tgv_tau(n0, u0), fields=lambda p: W.tgv_fields(p, n0, u0),
                    u_in=None, desc=desc, n0=n0, u0=u0, tgv=True)
    if name == "tgv32":
        n0, u0 = 32, 0.02
        spec = W.refined_box_mesh(stencil, 5, 8, 24)
        desc = f"{stencil} periodic Taylor-Green vortex, 32^3 coarse, central 16^3 refined"
        return dict(spec=spec, tau0=tgv_tau(n0, u0), fields=lambda p: W.tgv_fields(p, n0, u0),
                    u_in=None, desc=desc, n0=n0, u0=u0, tgv=True)
    if name == "tgv128":
        n0, u0 = 128, 0.01
        spec = W.refined_box_mesh(stencil, 7, 32, 96)
        desc = f"{stencil} periodic Taylor-Green vortex, 128^3 coarse, central 64^3 refined"
        return dict(spec=spec, tau0=tgv_tau(64, 0.02), fields=lambda p: W.tgv_fields(p, n0, u0),
                    u_in=None, desc=desc, n0=n0, u0=u0, tgv=True)
    if name == "sphere4":
        # the four-level configuration sized to one GPU's HBM: D = 128 finest
        # cells, boxes [-5D,19D]x[-5D,5D]^2, [-2.5D,9.5D]x[-2.5D,2.5D]^2,
        # [-1.25D,4.75D]x[-1.25D,1.25D]^2; about 449 M elements
        uin = 0.04
        spec = W.sphere_channel_mesh(128, 4, outlet="eq", stencil=stencil)
        tau_f = 0.5 + 3.0 * uin * 128 / 100.0
        tau0 = 0.5 + (tau_f - 0.5) / 8.0
        desc = (f"{stencil} channel [-15D,49D]x[-15D,15D]^2 with a sphere of D=128 finest "
                "cells, 4 nested levels, Re=100, free-stream equilibrium u=0.04 on all faces")
        return dict(spec=spec, tau0=tau0, u_in=[uin, 0.0, 0.0], uniform_u=[uin, 0.0, 0.0],
                    desc=desc, tgv=False)
    if name == "sphere3":
        uin = 0.04
        # free-stream equilibrium on every face: a zero-gradient (copy)
        # outlet destabilises BGK at the coarse level's tau = 0.507
        spec = W.sphere_channel_mesh(24, 3, outlet="eq", stencil=stencil)
        tau_f = 0.5 + 3.0 * uin * 24 / 100.0     # Re = u D / nu on the finest level
        tau0 = 0.5 + (tau_f - 0.5) / 4.0
        desc = (f"{stencil} channel [-15D,49D]x[-15D,15D]^2 with a sphere of D=24 finest "
                "cells, 3 nested levels, Re=100, free-stream equilibrium u=0.04 on all faces")
        return dict(spec=spec, tau0=tau0, u_in=[uin, 0.0, 0.0], uniform_u=[uin, 0.0, 0.0],
                    fields=lambda p: W.uniform_fields(len(p), 3, [uin, 0.0, 0.0]),
                    desc=desc, tgv=False)
    raise SystemExit(f"unknown workload {name}")


def weighted_updates(plan):
    """Fluid updates per coarse step: level k steps 2^k times (4^k under
    diffusive scaling, plans with four GhostFromCoarser layers)."""
    n_sub = 4 if plan.gfc_layers == 4 else 2
    return sum(plan.info[k]["n_fluid"] * n_sub ** k for k in range(plan.n_levels))


def make_plan(M, wl):
    if wl.get("diffusive"):
        M.set_gfc_layers(4)
    try:
        plan = M.Plan.from_spec(wl["spec"])
    finally:
        M.set_gfc_layers(2)
    if wl.get("walls"):
        spec = wl["spec"]
        plan.set_walls(*W.sphere_wall_links(spec, M.lattice(spec.stencil)[0]))
    return plan


def index_bytes_per_update(plan, k):
    """Bytes of the pull table read per updated element of level index k, as
    the device holds it: a 16-bit code per direction that is not a Morton
    direction of its block, the high halves for the blocks that need int32
    entries, and per 256 elements the block's header (4 int32) and bases
    (4 int32 per direction)."""
    q1 = plan.q - 1
    hdr = plan.export(k, "nbr_hdr").reshape(-1, 4).astype(np.int64)
    if not len(hdr):
        return 0.0
    mor = np.array([bin(v & 0xFFFFFFFF).count("1") for v in hdr[:, 0].tolist()])
    wide = hdr[:, 2] >= 0
    codes = 2.0 * (q1 - mor) + np.where(wide, 2.0 * q1, 0.0)
    return float(codes.mean()) + 16.0 * (q1 + 1) / 256.0


def make_sim(M, torch, wl, plan, precision):
    sim = M.Sim(plan, precision, wl["tau0"], u_in=wl["u_in"])
    dev = sim.device
    if wl.get("uniform_u") is not None:
        # uniform initial flow built on the device (S = 0); the inputs are
        # released after the fill to keep the HBM for the state
        for k in range(plan.n_levels):
            nf = plan.info[k]["n_fluid"]
            u = torch.empty((plan.d, nf), dtype=torch.float64, device=dev)
            for a in range(plan.d):
                u[a].fill_(wl["uniform_u"][a])
            sim.init(k, torch.ones(nf, dtype=torch.float64, device=dev), u, None)
        sim.fill_ghosts()
        torch.cuda.synchronize()
        sim.inputs = {}
        return sim
    for k in range(plan.n_levels):
        L = plan.level0 + k
        nf = plan.info[k]["n_fluid"]
        coords = plan.export(k, "coords")[:, :nf]
        pos = (coords.T.astype(np.float64) + 0.5) / float(1 << k)
        r, u, S = wl["fields"](pos)
        if plan.gfc_layers == 4:
            # diffusive scaling: level-k lattice units of velocity (u dt/dx),
            # density deviation (dt^2/dx^2) and strain rate (dt)
            f = 2.0 ** k
            r, u, S = 1.0 + (r - 1.0) / (f * f), u / f, S / (f * f)
        else:
            S = S * 2.0 ** -k
        idx = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]
        Sc = np.stack([S[:, a, b] for a, b in idx], 0)
        sim.init(k, torch.tensor(r, device=dev), torch.tensor(np.ascontiguousarray(u.T), device=dev),
                 torch.tensor(np.ascontiguousarray(Sc), device=dev))
    sim.fill_ghosts()
    return sim


def tgv_velocity_error(sim, plan, wl, t):
    """eps_u of u_x against the decayed closed form (Sec. 4.1 norm)."""
    nu0 = (wl["tau0"] - 0.5) / 3.0
    num = den = 0.0
    for k in range(plan.n_levels):
        nf = plan.info[k]["n_fluid"]
        coords = plan.export(k, "coords")[:, :nf]
        pos = (coords.T.astype(np.float64) + 0.5) / float(1 << k)
        _, ua, _ = W.tgv_fields(pos, wl["n0"], wl["u0"], nu0=nu0, t=t)
        us = sim.get_moments(k).cpu().numpy()[1]
        num += float(((us - ua[:, 0]) ** 2).sum())
        den += float((ua[:, 0] ** 2).sum())
    return math.sqrt(num / den)


def tgv_level_errors(sim, plan, n0, u0, tau0, t):
    """(eps_u, eps_S) of u_x and S_xx against the decayed closed form at
    coarse time t (Sec. 4.1 norm: unweighted over the fluid elements of all
    levels, S in coarsest-level units).  u is read as a moment of the
    stored state, S through the library's strain read-out (formed on the
    device from each element's pre-collision pdfs)."""
    nu0 = (tau0 - 0.5) / 3.0
    nu_num = nu_den = s_num = s_den = 0.0
    for k in range(plan.n_levels):
        nf = plan.info[k]["n_fluid"]
        coords = plan.export(k, "coords")[:, :nf]
        pos = (coords.T.astype(np.float64) + 0.5) / float(1 << k)
        _, ua, Sa = W.tgv_fields(pos, n0, u0, nu0=nu0, t=t)
        ux = sim.get_moments(k)[1].cpu().numpy()
        sxx = sim.get_strain(k)[0].cpu().numpy() * 2.0 ** k
        nu_num += float(((ux - ua[:, 0]) ** 2).sum())
        nu_den += float((ua[:, 0] ** 2).sum())
        s_num += float(((sxx - Sa[:, 0, 0]) ** 2).sum())
        s_den += float((Sa[:, 0, 0] ** 2).sum())
    return math.sqrt(nu_num / nu_den), math.sqrt(s_num / s_den)


def convergence_sweep(M, torch, bases=(32, 64, 128), precision="f64"):
    """Diffusive refinement of the two-level D3Q19 Taylor-Green box: coarse
    base N with the central half refined, u0 = 0.02 * 64 / N and tau0 fixed,
    run to t_D = 1 / (2 nu k^2) coarse steps; errors and observed orders."""
    tau0 = tgv_tau(64, 0.02)
    nu0 = (tau0 - 0.5) / 3.0
    rows = []
    for n0 in bases:
        level0 = int(round(math.log2(n0)))
        u0 = 0.02 * 64.0 / n0
        spec = W.refined_box_mesh("D3Q19", level0, n0 // 4, 3 * n0 // 4)
        plan = M.Plan.from_spec(spec)
        wl = dict(tau0=tau0, u_in=None, fields=lambda p, n0=n0, u0=u0: W.tgv_fields(p, n0, u0))
        sim = make_sim(M, torch, wl, plan, precision)
        k = 2.0 * math.pi / n0
        t_d = int(round(1.0 / (2.0 * nu0 * k * k)))
        print(f"[bench] sweep N={n0}: {t_d} coarse steps", file=sys.stderr, flush=True)
        ms = timed_steps(torch, sim, t_d)
        eu, es = tgv_level_errors(sim, plan, n0, u0, tau0, t_d)
        rows.append(dict(base=n0, u0=u0, coarse_steps=t_d, eps_u=eu, eps_S=es,
                         seconds=round(ms / 1e3, 2), status=sim.status()))
        del sim
    for a, b in zip(rows, rows[1:]):
        b["order_u"] = math.log(a["eps_u"] / b["eps_u"], 2)
        b["order_S"] = math.log(a["eps_S"] / b["eps_S"], 2)
    return {"precision": precision, "tau0": tau0, "refinement": "central half refined once",
            "results": rows}


def timed_steps(torch, sim, steps):
    s = sim.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    sim.step(steps)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def _dir_perm(c_lib, c_oracle):
    return [int(np.where((c_oracle == c_lib[i]).all(1))[0][0]) for i in range(len(c_lib))]


def oracle_accuracy(wl, steps, gpu_pdfs, lattice):
    """The FP64 oracle on the host for `steps` coarse steps from the
    workload's initial state; for each precision in `gpu_pdfs` ({precision:
    list of (treeids, [q][n_fluid] post-collision pdfs) per level, taken
    after the same number of steps}) the max relative pdf difference."""
    import torch
    from oracle import mesh as omesh
    from oracle import solver as osolver
    om = omesh.build(wl["spec"])
    sim = osolver.OracleSim(om, wl["tau0"], u_in=None if wl["u_in"] is None
                            else torch.tensor(wl["u_in"], dtype=torch.float64))
    rho, u, S = {}, {}, {}
    for L in range(om.level0, om.lmax + 1):
        pos = om.positions(L)[:om.lev(L).n_fluid]
        r, uu, SS = wl["fields"](pos)
        rho[L], u[L], S[L] = r, uu, SS * 2.0 ** -(L - om.level0)
    sim.init(rho, u, S)
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    perm = _dir_perm(lattice, np.asarray(sim.lat.c))
    errs = {}
    for prec, levels in gpu_pdfs.items():
        worst = 0.0
        for k, (tid, g) in enumerate(levels):
            lev = om.lev(om.level0 + k)
            ot = np.asarray(lev.tid)
            order = np.argsort(ot)
            g2o = order[np.searchsorted(ot[order], tid)]
            o = sim.post_collision(om.level0 + k).detach().numpy()[perm][:, g2o]
            worst = max(worst, float((np.abs(g - o) / np.abs(o)).max()))
        errs[prec] = worst
    return errs, dt


def cpu_baseline(stencil, sample_d, steps):
    """The FP64 oracle as it stands, on one host thread, on a bounded sample
    of the four-level sphere workload: the same channel, nesting boxes,
    Reynolds number and inflow with the sphere resolved by `sample_d`
    finest cells instead of 128, for `steps` coarse steps from the uniform
    free stream.  MLUPS with the same weighted count as the GPU figure."""
    import torch
    from oracle import mesh as omesh
    from oracle import solver as osolver
    uin = 0.04
    spec = W.sphere_channel_mesh(sample_d, 4, outlet="eq", stencil=stencil)
    tau_f = 0.5 + 3.0 * uin * sample_d / 100.0
    nthreads = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        om = omesh.build(spec)
        t_build = time.perf_counter() - t0
        sim = osolver.OracleSim(om, 0.5 + (tau_f - 0.5) / 8.0,
                                u_in=torch.tensor([uin, 0.0, 0.0], dtype=torch.float64))
        rho, u, S = {}, {}, {}
        for L in range(om.level0, om.lmax + 1):
            rho[L], u[L], S[L] = W.uniform_fields(om.lev(L).n_fluid, 3, [uin, 0.0, 0.0])
        sim.init(rho, u, S)
        t1 = time.perf_counter()
        sim.step(steps)
        dt = time.perf_counter() - t1
    finally:
        torch.set_num_threads(nthreads)
    upd = sum(om.lev(L).n_fluid << (L - om.level0) for L in range(om.level0, om.lmax + 1))
    n = sum(om.lev(L).n for L in range(om.level0, om.lmax + 1))
    return dict(value=round(upd * steps / dt / 1e6, 4), unit="MLUPS", cores=1, kind="oracle",
                sample=f"{stencil} four-level sphere channel of the same geometry with D = "
                       f"{sample_d} finest cells ({n:,} elements, {upd:,} weighted updates per "
                       f"coarse step), {steps} coarse steps from the uniform free stream: "
                       f"{dt:.1f} s wall on one thread (FP64, torch CPU ops; mesh analysis "
                       f"{t_build:.1f} s not counted), "
                       f"{platform.processor() or platform.machine()}, "
                       f"{os.cpu_count()} logical CPUs visible")


def fluid_pdfs(sim, plan):
    """Per level: (treeIDs, [q][n_fluid] FP64 post-collision pdfs) on the host."""
    res = []
    for k in range(plan.n_levels):
        nf = plan.info[k]["n_fluid"]
        res.append((plan.export(k, "treeid")[:nf], sim.get_pdf(k)[:, :nf].cpu().numpy()))
    return res


def drag_inflow_gradient(M, torch, sim, uin, n_steps, K, snapshots):
    """Gradient of the x drag after n_steps coarse steps with respect to the
    free-stream velocity `uin`, which sets the EQ faces and the uniform
    initial field: forward with a checkpoint every K coarse steps, each
    segment reversed last first (recursive bisection with at most
    `snapshots` extra states), then the initialisation reversed."""
    from paper_1601_06984_amd import autograd as AG
    ev = lambda: torch.cuda.Event(enable_timing=True)
    e0, e1, e2 = ev(), ev(), ev()
    ck = {}
    torch.cuda.synchronize()
    e0.record(sim.stream)
    t = 0
    while t < n_steps:
        ck[t] = sim.save_checkpoint()
        m = min(K, n_steps - t)
        sim.step(m)
        t += m
    J = float(sim.diagnostics(M.DIAG_FORCE)[0])
    e1.record(sim.stream)
    if getattr(sim, "adj_workspace", None) is None:
        sim.adjoint_attach()
    sim.adjoint_seed("drag_x")
    if snapshots == "auto":
        snapshots = AG.snapshot_budget(sim)
    for start in sorted(ck, reverse=True):
        print(f"[bench] reversing coarse steps {start}..{min(start + K, n_steps)}",
              file=sys.stderr, flush=True)
        AG.reverse_steps(sim, ck[start], min(K, n_steps - start), snapshots)
        torch.cuda.synchronize()
    # the run starts from the uniform free stream u0 = u_in: its initial
    # field is a second path from u_in to the drag
    rho0, u0 = [], []
    for k in range(sim.plan.n_levels):
        nf = sim.plan.info[k]["n_fluid"]
        rho0.append(torch.ones(nf, dtype=torch.float64, device=sim.device))
        u = torch.empty((sim.plan.d, nf), dtype=torch.float64, device=sim.device)
        for a in range(sim.plan.d):
            u[a].fill_(uin[a])
        u0.append(u)
    du = sim.adjoint_init(rho0, u0, None)
    via_init = [sum(float(g[a].sum()) for g in du) for a in range(sim.plan.d)]
    del rho0, u0, du
    dtau, domega, duin = sim.adjoint_params()
    e2.record(sim.stream)
    torch.cuda.synchronize()
    return {"coarse_steps": n_steps, "checkpoint_every": K, "max_snapshots": snapshots,
            "drag_x": J, "dJ_du_in_faces": list(duin[:3]),
            "dJ_du_in_via_initial_field": via_init,
            "dJ_du_in": [duin[a] + via_init[a] for a in range(sim.plan.d)], "dJ_dtau0": dtau,
            "forward_ms": round(e0.elapsed_time(e1), 1),
            "backward_ms": round(e1.elapsed_time(e2), 1),
            "backward_ms_per_coarse_step": round(e1.elapsed_time(e2) / n_steps, 2),
            "peak_device_GB": round(torch.cuda.max_memory_allocated() / 1e9, 1)}


def _say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def working_set_bytes(plan, prec):
    """Device bytes one coarse step streams through: both pdf arrays and the
    pull table of every level."""
    q = plan.q
    tot = 0
    for k in range(plan.n_levels):
        n = plan.info[k]["n"]
        tot += 2 * q * n * STORAGE_BYTES[prec] + int(index_bytes_per_update(plan, k) * n)
    return tot


def forward_leg(M, torch, wl, plan, prec, steps, warmup):
    """Timed coarse steps (graph replay) and per-level stream-collide
    durations (direct launches bracketed by events on the bound stream)."""
    upd = weighted_updates(plan)
    sim = make_sim(M, torch, wl, plan, prec)
    _say(f"{prec}: warmup {warmup}")
    sim.step(warmup)
    torch.cuda.synchronize()
    _say(f"{prec}: timed {steps} coarse steps")
    ms = timed_steps(torch, sim, steps)
    _say(f"{prec}: kernel timing over {steps} coarse steps")
    sim.profile(True)
    ms_direct = timed_steps(torch, sim, steps)
    sim.profile(False)
    q = plan.q
    alg = algorithmic_bytes(q, prec)
    prof = []
    for k in range(plan.n_levels):
        kms, n, el = sim.profile_read(k)
        asr = 2 * q * STORAGE_BYTES[prec] + index_bytes_per_update(plan, k)
        t = kms / 1e3
        prof.append(dict(level=plan.level0 + k, launches=n, ms_total=round(kms, 4),
                         us_per_launch=round(1e3 * kms / max(n, 1), 2),
                         elements_per_launch=round(el / max(n, 1), 1),
                         algorithmic_gbs=round(el * alg / 1e9 / t, 1) if t else 0.0,
                         as_read_bytes_per_update=round(asr, 2),
                         as_read_gbs=round(el * asr / 1e9 / t, 1) if t else 0.0))
    dom = max(prof, key=lambda p: p["ms_total"])
    return sim, dict(value=upd * steps / (ms / 1e3) / 1e6, ms=ms, ms_direct=ms_direct,
                     kernels=prof, dominant=dom, status=sim.status())


def adjoint_leg(torch, sim, plan, prec, n_adj):
    """Reverse coarse steps (tape rerun + transposed kernels) and per-level
    reverse stream-collide durations."""
    upd = weighted_updates(plan)
    sim.adjoint_attach()
    ck = sim.save_checkpoint()
    sim.adjoint_seed("ke")
    for _ in range(2):
        sim.adjoint_step(ck)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    for _ in range(n_adj):
        sim.adjoint_step(ck)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    adj_ms = e0.elapsed_time(e1) / n_adj
    sim.profile(True)
    for _ in range(n_adj):
        sim.adjoint_step(ck)
    torch.cuda.synchronize()
    sim.profile(False)
    q = plan.q
    alg = algorithmic_bytes_adjoint(q, prec)
    akern = []
    for k in range(plan.n_levels):
        kms, n, el = sim.profile_read(k, kind=1)
        t = kms / 1e3
        akern.append(dict(level=plan.level0 + k, launches=n, ms_total=round(kms, 4),
                          us_per_launch=round(1e3 * kms / max(n, 1), 2),
                          elements_per_launch=round(el / max(n, 1), 1),
                          algorithmic_gbs=round(el * alg / 1e9 / t, 1) if t else 0.0))
    adom = max(akern, key=lambda p: p["ms_total"])
    fwd_ms = None
    del ck
    return {
        "ms_per_step": round(adj_ms, 4),
        "mlups": round(upd / (adj_ms / 1e3) / 1e6, 1),
        "note": "one reverse coarse step = tape rerun of the forward step + transposed kernels",
        "kernel": f"k_adj_sc level {adom['level']} ({prec} state, "
                  f"{'FP64' if prec == 'f64' else 'FP32'} lambda)",
        "algorithmic_bytes_per_update": alg,
        "achieved_gbs": adom["algorithmic_gbs"],
        "frac": round(adom["algorithmic_gbs"] / HBM_PEAK_GBS, 4),
        "kernels": akern,
        "forward_ms_per_step": fwd_ms,
    }


def precision_study(M, torch, n_fix, n_chk, with_oracle, name="tgv64"):
    """Fixed-error study on a two-level D3Q19 Taylor-Green box (tgv64: 64^3
    with the central 32^3 refined, cache resident; tgv128: 128^3 with the
    central 64^3 refined, 0.9 GB, HBM bound): MLUPS and eps_u after n_fix
    coarse steps for F64, F32 and F16S; with the oracle, the pdfs after
    n_chk steps against the FP64 oracle."""
    wl = workload(name)
    plan = M.Plan.from_spec(wl["spec"])
    upd = weighted_updates(plan)
    study, gpu_pdfs = {}, {}
    for p in ("f64", "f32", "f16s"):
        _say(f"precision study {p}")
        s2 = make_sim(M, torch, wl, plan, p)
        done = 0
        if with_oracle and 0 < n_chk <= n_fix - 20:
            s2.step(n_chk)
            gpu_pdfs[p] = fluid_pdfs(s2, plan)
            done = n_chk
        s2.step(20)
        done += 20
        t_ms = timed_steps(torch, s2, n_fix - done)
        study[p] = dict(mlups=round(upd * (n_fix - done) / (t_ms / 1e3) / 1e6, 1),
                        eps_u=tgv_velocity_error(s2, plan, wl, n_fix), status=s2.status(),
                        working_set_bytes=working_set_bytes(plan, p))
        del s2
    ref = study["f64"]["eps_u"]
    for p in study:
        study[p]["eps_u_vs_f64"] = round(study[p]["eps_u"] / ref, 4)
        study[p]["fixed_error_pass"] = bool(study[p]["eps_u"] <= 1.05 * ref)
    out = {"workload": wl["desc"], "coarse_steps": n_fix,
           "fixed_error_bar": "eps_u <= 1.05 x eps_u(F64)", "results": study}
    if gpu_pdfs:
        _say(f"oracle accuracy check: {n_chk} coarse steps")
        c, _ = M.lattice(plan.stencil)
        errs, dt = oracle_accuracy(wl, n_chk, gpu_pdfs, np.asarray(c))
        for p, e in errs.items():
            study[p][f"max_rel_pdf_err_vs_oracle_{n_chk}"] = e
        out["oracle_seconds"] = round(dt, 1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sphere4")
    ap.add_argument("--precision", default="f16s", choices=["f64", "f32", "f16s"])
    ap.add_argument("--variants", type=int, default=1,
                    help="also time the other storage precision (F32 for F16S and back) on "
                         "the same mesh")
    ap.add_argument("--study", type=int, default=1,
                    help="run the fixed-error precision study on the two-level TGV box")
    ap.add_argument("--cpu-steps", type=int, default=100,
                    help="coarse steps of the oracle accuracy check in the precision study")
    ap.add_argument("--cpu-sample-d", type=int, default=16,
                    help="sphere diameter (finest cells) of the oracle's timing sample")
    ap.add_argument("--cpu-sample-steps", type=int, default=10)
    ap.add_argument("--drag-steps", type=int, default=0,
                    help="sphere workloads: run this many coarse steps in F32 and F16S "
                         "from the initial state and report the drag coefficient")
    ap.add_argument("--adjoint", type=int, default=10,
                    help="time this many reverse coarse steps (0: skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-ceiling", type=int, default=1,
                    help="also time a plain 2 GiB device copy (read + write)")
    ap.add_argument("--drag-adjoint", type=int, default=0,
                    help="sphere workloads: dJ/du_in of the x drag over this many coarse steps")
    ap.add_argument("--checkpoint-every", type=int, default=50)
    ap.add_argument("--snapshots", type=int, default=-1,
                    help="extra states kept while reversing a segment "
                         "(-1: as many as the free device memory holds)")
    ap.add_argument("--sweep", type=int, default=0,
                    help="also run the FP64 convergence sweep (bases 32/64/128 to t_D)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a plain device copy of this size (counter calibration)")
    ap.add_argument("--calib-gather-mib", type=int, default=0,
                    help="gather 2-byte values at random positions of a buffer of this size "
                         "(counter calibration for partial-line reads)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        raise SystemExit(2)

    import torch
    import paper_1601_06984_amd as M
    torch.cuda.set_device(0)
    wl = workload(args.workload)
    _say(f"workload {args.workload}: planning")
    t0 = time.perf_counter()
    plan = make_plan(M, wl)
    t_plan = time.perf_counter() - t0
    upd = weighted_updates(plan)
    prec = args.precision
    sim, fw = forward_leg(M, torch, wl, plan, prec, args.steps, args.warmup)
    q = plan.q
    dom = fw["dominant"]
    alg = algorithmic_bytes(q, prec)
    t_launch = dom["us_per_launch"] * 1e-6
    achieved = dom["algorithmic_gbs"]
    ws = working_set_bytes(plan, prec)
    traffic = measured_traffic(args.workload, prec, dom["level"])
    roof = {"bound": "hbm" if ws > INFINITY_CACHE_BYTES else "infinity_cache",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": f"k_stream_collide level {dom['level']} ({prec})",
            "algorithmic_bytes_per_update": alg,
            "algorithmic_bytes_note": f"2 q S + 4 (q-1): q = {q} pdfs read and written at "
                                      f"{STORAGE_BYTES[prec]} B, an int32 pull index per "
                                      "moving direction",
            "elements_per_launch": dom["elements_per_launch"],
            "algorithmic_bytes_per_launch": round(dom["elements_per_launch"] * alg),
            "us_per_launch": dom["us_per_launch"],
            "working_set_bytes": ws,
            "as_read_bytes_per_update": dom["as_read_bytes_per_update"],
            "as_read_frac": round(dom["as_read_gbs"] / HBM_PEAK_GBS, 4),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated); null when the kernel sources changed since"}
    if traffic:
        roof["traffic_gbs"] = round(traffic / t_launch / 1e9, 1)
        roof["traffic_frac"] = round(traffic / t_launch / 1e9 / HBM_PEAK_GBS, 4)
        roof["traffic_over_algorithmic"] = round(traffic / (dom["elements_per_launch"] * alg), 3)
        roof["traffic_over_as_read"] = round(
            traffic / (dom["elements_per_launch"] * dom["as_read_bytes_per_update"]), 3)
    out = {
        "metric": METRIC, "value": round(fw["value"], 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": fw["ms"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "f64" else "f32", "data": "synthetic",
        "config": {"workload": wl["desc"], "name": args.workload,
                   "storage": {"f64": "FP64", "f32": "FP32",
                               "f16s": "FP16 shifted deviations, per-level scale"}[prec],
                   "collision": "FP64" if prec == "f64" else "FP32",
                   "elements": int(sum(i["n"] for i in plan.info)),
                   "weighted_updates_per_step": int(upd), "levels": plan.n_levels,
                   "planning_s": round(t_plan, 1)},
        "roofline": roof,
        "kernels": fw["kernels"],
        "ms_per_step_direct_launches": fw["ms_direct"] / args.steps,
        "status_flags": fw["status"],
    }
    if args.adjoint and plan.gfc_layers == 4:
        out["adjoint"] = {"note": "the adjoint covers acoustic scaling only"}
    elif args.adjoint:
        _say(f"adjoint: {args.adjoint} reverse coarse steps")
        out["adjoint"] = adjoint_leg(torch, sim, plan, prec, args.adjoint)
        out["adjoint"]["forward_ms_per_step"] = round(fw["ms"] / args.steps, 4)
        out["adjoint"]["reverse_over_forward"] = round(
            out["adjoint"]["ms_per_step"] / (fw["ms"] / args.steps), 3)
    sim = None
    import gc
    gc.collect()
    torch.cuda.empty_cache()
    if args.variants:
        other = "f32" if prec == "f16s" else "f16s"
        s2, fw2 = forward_leg(M, torch, wl, plan, other, args.steps, args.warmup)
        d2 = fw2["dominant"]
        a2 = algorithmic_bytes(q, other)
        out["precision_variants"] = {other: {
            "mlups": round(fw2["value"], 2), "ms_per_step": fw2["ms"] / args.steps,
            "kernel": f"k_stream_collide level {d2['level']} ({other})",
            "algorithmic_bytes_per_update": a2, "achieved_gbs": d2["algorithmic_gbs"],
            "frac": round(d2["algorithmic_gbs"] / HBM_PEAK_GBS, 4),
            "us_per_launch": d2["us_per_launch"], "status_flags": fw2["status"]},
            prec: {"mlups": out["value"]}}
        out["precision_variants"]["speedup_f16s_over_f32"] = round(
            (out["value"] / fw2["value"]) if prec == "f16s" else (fw2["value"] / out["value"]), 3)
        del s2
        gc.collect()
        torch.cuda.empty_cache()
    if args.drag_adjoint and not wl.get("tgv"):
        _say(f"drag gradient over {args.drag_adjoint} coarse steps")
        sim2 = make_sim(M, torch, wl, plan, prec)
        out["drag_adjoint"] = drag_inflow_gradient(
            M, torch, sim2, wl["uniform_u"], args.drag_adjoint, args.checkpoint_every,
            "auto" if args.snapshots < 0 else args.snapshots)
        del sim2
        gc.collect()
        torch.cuda.empty_cache()
    if args.drag_steps and not wl.get("tgv"):
        D = wl["spec"].meta["D"]
        uin = wl["u_in"][0]
        drag = {}
        for p in ("f32", "f16s"):
            _say(f"drag run {p}: {args.drag_steps} coarse steps")
            s3 = make_sim(M, torch, wl, plan, p)
            hist = []
            chunk = max(1, args.drag_steps // 10)
            t_ms = 0.0
            done = 0
            while done < args.drag_steps:
                m = min(chunk, args.drag_steps - done)
                t_ms += timed_steps(torch, s3, m)
                done += m
                fx = float(s3.diagnostics(M.DIAG_FORCE)[0])
                hist.append((done, round(2.0 * fx / (uin ** 2 * math.pi * D * D / 4.0), 5)))
            drag[p] = dict(c_d=hist[-1][1], c_d_history=hist,
                           mlups=round(upd * args.drag_steps / (t_ms / 1e3) / 1e6, 1),
                           status=s3.status())
            del s3
        out["drag"] = {"coarse_steps": args.drag_steps, "D_finest": D, "u_in": uin,
                       "definition": "c_D = 2 F_x / (rho0 u_in^2 pi D^2 / 4), finest-level units",
                       "results": drag}
    plan = None
    gc.collect()
    if args.study:
        out["precision_study"] = precision_study(M, torch, 1000, args.cpu_steps,
                                                 not args.no_cpu)
        gc.collect()
        torch.cuda.empty_cache()
        # the same study where the working set exceeds the Infinity Cache
        out["precision_study_hbm"] = precision_study(M, torch, 1000, 0, False, "tgv128")
    if args.sweep:
        out["convergence"] = convergence_sweep(M, torch)
    if args.copy_ceiling:
        # practical streaming ceiling of this device: a plain 2 GiB copy
        n = 2 << 30
        a_ = torch.empty(n, dtype=torch.uint8, device="cuda")
        b_ = torch.empty_like(a_)
        b_.copy_(a_)
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(5):
            b_.copy_(a_)
        c1.record()
        torch.cuda.synchronize()
        out["copy_ceiling_gbs"] = round(2 * n * 5 / (c0.elapsed_time(c1) / 1e3) / 1e9, 1)
        del a_, b_
    if args.calib_copy_mib:
        n = args.calib_copy_mib << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = n
    if args.calib_gather_mib:
        out["calib_gather"] = calib_gather(torch, args.calib_gather_mib << 20)
    if not args.no_cpu:
        _say(f"cpu baseline (oracle, one thread): D = {args.cpu_sample_d} sample")
        stencil = wl["spec"].stencil if not wl.get("tgv") else "D3Q19"
        out["cpu_baseline"] = cpu_baseline(stencil, args.cpu_sample_d, args.cpu_sample_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
