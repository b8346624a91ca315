"""GPU parity on the degenerate and boundary-sized meshes of the method.

* Single-level periodic boxes whose element count is below one pull-table
  block (64 elements: one partial work-group, per-lane stores), exactly one
  block (256) or exactly two (512: whole work-groups only, every store
  through the LDS tile, the last block included).  No ghosts, no fills:
  the schedule reduces to the plain stream-collide of Eq. bgk, and FP64
  mass is conserved to rounding.
* Two-level meshes with the smallest refined patch the ghost rules allow
  (two by two coarse cells in 2D, 2^3 in 3D), where every fine fluid
  element (2D) or every second one (3D) is an interpolation source and
  most elements of the fine level are GhostFromCoarser: the fills and the
  capture tail are most of the level.

Every case runs the oracle on the same seeded Taylor-Green input and
compares all post-collision pdfs, ghosts included: F64 1e-12, F32 1e-5,
F16S 2e-3 (relative).
"""
import sys

import pytest
import torch

import workloads as W
from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f16s": 2e-3}


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1601_06984_amd  # noqa: F401  (fails loudly if not built)


@pytest.mark.parametrize("stencil,level", [("D2Q9", 3), ("D2Q9", 4), ("D3Q19", 2),
                                           ("D3Q19", 3), ("D3Q27", 2)])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_single_level_boxes_around_one_block(stencil, level, prec):
    import paper_1601_06984_amd as M
    spec = W.uniform_box_mesh(stencil, level)
    n0 = 1 << level
    _say("single level", stencil, n0, prec)
    fields = H.tgv(n0, 0.03)
    osim = H.oracle_run(spec, 0.7, fields, 20)
    sim = H.gpu_sim(spec, prec, 0.7, fields)
    assert sim.plan.info[0]["n"] == n0 ** sim.plan.d
    m0 = float(sim.diagnostics(M.DIAG_MASS).cpu()[0])
    sim.step(20)
    err = H.compare_post(sim, osim)
    assert err < TOL[prec], err
    assert sim.status() == 0
    if prec == "f64":
        m1 = float(sim.diagnostics(M.DIAG_MASS).cpu()[0])
        assert abs(m1 - m0) <= 1e-13 * abs(m0)


@pytest.mark.parametrize("stencil,level0,lo,hi", [("D2Q9", 3, 2, 4), ("D2Q9", 4, 7, 9),
                                                  ("D3Q19", 3, 2, 4), ("D3Q27", 3, 2, 4)])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_smallest_refined_patch(stencil, level0, lo, hi, prec):
    spec = W.refined_box_mesh(stencil, level0, lo, hi)
    n0 = 1 << level0
    _say("smallest refined patch", stencil, n0, lo, hi, prec)
    fields = H.tgv(n0, 0.03)
    osim = H.oracle_run(spec, 0.7, fields, 10)
    sim = H.gpu_sim(spec, prec, 0.7, fields)
    info = sim.plan.info[1]
    # every fine fluid element is a GhostFromFiner source in 2D (all four
    # children), every second one in 3D (four of the eight children)
    assert info["n_cap_fluid"] * (2 if sim.plan.d == 3 else 1) == info["n_fluid"]
    sim.step(10)
    err = H.compare_post(sim, osim)
    assert err < TOL[prec], err
    assert sim.status() == 0
