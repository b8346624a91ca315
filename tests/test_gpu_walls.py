"""Curved walls (linear interpolated bounce-back, Sec. 2.3) on the GPU
against the oracle: the plane channel whose wall position the oracle pins
follow from the fractions, and the sphere with the fractions at which its
surface cuts each link; state and momentum-exchange force.

Tolerances as for the other forward parity tests: F64 1e-12 relative per
pdf, F32 1e-5 (a few ulp of O(1) pdfs over the steps run), F16S 3e-3
(2^-11 storage rounding of the deviations, accumulated).
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import mesh as omesh
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1601_06984_amd  # noqa: F401


TOL = {"f64": 1e-12, "f32": 1e-5, "f16s": 3e-3}


def _both(spec, links_of):
    """The same links in each side's direction order."""
    import paper_1601_06984_amd as M
    om = omesh.build(spec)
    c_lib, _ = M.lattice(spec.stencil)
    return om, links_of(c_lib), links_of(om.lattice.c)


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("q_low,q_high", [(0.2, 0.7), (0.9, 0.35), (0.0, 1.0)])
@pytest.mark.parametrize("precision", ["f64", "f32", "f16s"])
def test_channel_walls_match_oracle(stencil, q_low, q_high, precision):
    import paper_1601_06984_amd as M
    h = 24
    spec = W.plane_channel_mesh(stencil, 5, 4, h)
    om, lw, ow = _both(spec, lambda c: W.plane_wall_links(spec, c, q_low, q_high))
    z_lo = 1.5 - q_low
    H_ = (h - 1.5 + q_high) - z_lo
    fields = lambda pos: W.shear_wave_fields(pos, z_lo, H_, 0.05)
    _say("channel", stencil, q_low, q_high, precision)
    steps = 40
    osim = H.oracle_run(spec, 0.8, fields, steps, om=om, walls=ow)
    plan = M.Plan.from_spec(spec)
    plan.set_walls(*lw)
    assert plan.info[0]["n_wall"] == len(lw[0])
    sim = H.gpu_sim(spec, precision, 0.8, fields, plan=plan)
    sim.step(steps)
    assert H.compare_post(sim, osim) < TOL[precision]


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("q_low,q_high", [(0.7, 0.8), (0.3, 0.6)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_single_row_between_walls(stencil, q_low, q_high, precision):
    """One fluid row between two walls: every element has links into both,
    so a link with q >= 1/2 reads the entry its opposite link's value goes
    to, and a link with q < 1/2 has no second element (halfway rule)."""
    import paper_1601_06984_amd as M
    spec = W.plane_channel_mesh(stencil, 5, 4, 3)
    om, lw, ow = _both(spec, lambda c: W.plane_wall_links(spec, c, q_low, q_high))
    d = spec.dim
    fields = lambda pos: W.uniform_fields(len(pos), d, [0.03] + [0.0] * (d - 1))
    _say("single row", stencil, q_low, q_high, precision)
    osim = H.oracle_run(spec, 0.8, fields, 4, om=om, walls=ow)
    plan = M.Plan.from_spec(spec)
    plan.set_walls(*lw)
    sim = H.gpu_sim(spec, precision, 0.8, fields, plan=plan)
    sim.step(4)
    assert H.compare_post(sim, osim) < TOL[precision]


def _sphere_small(stencil):
    return W.sphere_channel_mesh(8, 2, l0_per_d=4, length=(-2.0, 3.0), half_width=2.0,
                                 boxes_in_d=((-1.0, 1.5, 1.0),), stencil=stencil)


@pytest.mark.parametrize("stencil", ["D3Q19", "D3Q27"])
@pytest.mark.parametrize("precision", ["f64", "f32", "f16s"])
def test_sphere_walls_and_drag_match_oracle(stencil, precision):
    """Sphere in a channel (EQ inflow and sides, copy outlet) with the
    fractions at which the sphere cuts each link; the drag follows the
    interpolated returning values."""
    import paper_1601_06984_amd as M
    spec = _sphere_small(stencil)
    om, lw, ow = _both(spec, lambda c: W.sphere_wall_links(spec, c))
    uin = np.array([0.04, 0.0, 0.0])
    fields = lambda pos: W.uniform_fields(len(pos), 3, uin)
    _say("sphere walls", stencil, precision)
    steps = 30
    osim = H.oracle_run(spec, 0.6, fields, steps, u_in=uin, om=om, walls=ow)
    plan = M.Plan.from_spec(spec)
    plan.set_walls(*lw)
    sim = H.gpu_sim(spec, precision, 0.6, fields, u_in=uin, plan=plan)
    sim.step(steps)
    tol = TOL[precision]
    assert H.compare_post(sim, osim) < tol
    d = sim.diagnostics(M.DIAG_FORCE).cpu().numpy()[:3]   # Fx, Fy, Fz
    F = osim.force().numpy()
    assert F[0] > 0
    assert np.allclose(d, F, rtol=tol * 100, atol=tol * 10), (d, F)
    # the fractions change the answer: halfway bounce-back gives another force
    osim_h = H.oracle_run(spec, 0.6, fields, steps, u_in=uin, om=om)
    assert abs(float(osim_h.force()[0]) - F[0]) > 1e-3 * abs(F[0])


def test_walls_across_graph_replays_and_grouped_launches():
    """Two levels with walls on the finest, stepped with captured graphs
    (two coarse steps per replay) and eagerly: same bits."""
    import paper_1601_06984_amd as M
    spec = _sphere_small("D3Q19")
    lw = W.sphere_wall_links(spec, M.lattice("D3Q19")[0])
    uin = np.array([0.04, 0.0, 0.0])
    fields = lambda pos: W.uniform_fields(len(pos), 3, uin)
    _say("sphere walls graphs")
    out = []
    for graphs in (False, True):
        plan = M.Plan.from_spec(spec)
        plan.set_walls(*lw)
        sim = H.gpu_sim(spec, "f32", 0.6, fields, u_in=uin, plan=plan)
        sim.use_graphs(graphs)
        for _ in range(3):
            sim.step(4)
            torch.cuda.synchronize()
        out.append([sim.get_pdf(k) for k in range(plan.n_levels)])
    for a, b in zip(*out):
        assert torch.equal(a, b)


def test_checkpoints_with_walls():
    """The wall pre-pass writes into the state a stream-collide consumes;
    saved checkpoints and restarts stay exact, and a reverse step leaves the
    checkpoint it reads untouched (its level with walls works on a copy)."""
    import paper_1601_06984_amd as M
    spec = _sphere_small("D3Q19")
    lw = W.sphere_wall_links(spec, M.lattice("D3Q19")[0])
    uin = np.array([0.04, 0.0, 0.0])
    fields = lambda pos: W.uniform_fields(len(pos), 3, uin)
    _say("sphere walls checkpoints")
    plan = M.Plan.from_spec(spec)
    plan.set_walls(*lw)
    sim = H.gpu_sim(spec, "f32", 0.6, fields, u_in=uin, plan=plan)
    sim.step(5)
    ck = sim.save_checkpoint()
    sim.step(5)
    a = [sim.get_pdf(k) for k in range(plan.n_levels)]
    sim.load_checkpoint(ck)
    sim.step(5)
    b = [sim.get_pdf(k) for k in range(plan.n_levels)]
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    # reverse step from the checkpoint, twice: same result, checkpoint kept
    sim.load_checkpoint(ck)
    sim.step(1)
    sim.adjoint_attach()
    before = ck.clone()
    out = []
    for _ in range(2):
        sim.adjoint_seed("drag_x")
        sim.adjoint_step(ck)
        torch.cuda.synchronize()
        assert torch.equal(ck, before)
        out.append([sim.adjoint_lambda(k).clone() for k in range(plan.n_levels)])
    for x, y in zip(*out):
        assert torch.equal(x, y)
