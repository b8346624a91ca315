"""The no-allocation diagnostics entry point against mlbm_diagnostics.

mlbm_diagnostics_noalloc keeps its per-block partials in the library's
static scratch array instead of the simulation's workspace; it must give
the same FP64 reductions (mass, kinetic energy, momentum-exchange force)
bit for bit, call after call, with a smaller mesh after a larger one (the
scratch keeps the last call's contents).
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_noalloc_diagnostics_equal_workspace_diagnostics():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1601_06984_amd as M
    mask = M.DIAG_MASS | M.DIAG_KE | M.DIAG_FORCE
    cases = [
        # larger first: a three-level sphere channel with bounce-back links
        ("sphere D=16, 3 levels, f32",
         lambda: W.sphere_channel_mesh(16, 3, outlet="eq"), "f32", 0.52, [0.04, 0.0, 0.0]),
        # then a smaller two-level box
        ("TGV box 16^3 + 8^3, f64",
         lambda: W.refined_box_mesh("D3Q19", 4, 4, 12), "f64", 0.6, None),
    ]
    sizes = []
    for name, spec_fn, prec, tau0, uin in cases:
        _say("no-alloc diagnostics:", name)
        spec = spec_fn()
        if uin is None:
            fields = H.tgv(16, 0.03)
        else:
            fields = lambda p, uin=uin: W.uniform_fields(len(p), 3, uin)
        sim = H.gpu_sim(spec, prec, tau0, fields, u_in=uin)
        sim.step(3)
        sizes.append(sum(i["n"] for i in sim.plan.info))
        out_a = torch.full((5,), float("nan"), dtype=torch.float64, device=sim.device)
        out_b = torch.full((5,), float("nan"), dtype=torch.float64, device=sim.device)
        for _ in range(2):
            sim.diagnostics(mask, out_a)
            sim.diagnostics_noalloc(mask, out_b)
            torch.cuda.synchronize()
            a, b = out_a.cpu().numpy(), out_b.cpu().numpy()
            assert np.isfinite(a).all()
            assert np.array_equal(a, b), (a, b)
            sim.step(1)
        if uin is not None:
            assert abs(a[2]) > 0          # the force is exercised
        assert sim.status() == 0
        del sim
    assert sizes[1] < sizes[0]
