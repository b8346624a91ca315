"""Second-order convergence of the multilevel GPU path (FP64) on the
two-level D3Q19 Taylor-Green box under diffusive refinement, measured at
t_D against the closed-form decay (Sec. 4.1; the paper reports second
order for u and S but prints no values)."""
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_tgv_velocity_and_strain_converge_at_second_order():
    """Bases 32, 64 and 128 (central half refined, u0 = 0.04 / 0.02 / 0.01,
    tau fixed, 6,366 / 25,465 / 101,859 coarse steps to t_D).  Measured on
    MI355X: orders 1.78 (u) and 1.85 (S) between 32 and 64, 1.84 and 1.90
    between 64 and 128; the order approaches 2 under refinement."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import bench
    import paper_1601_06984_amd as M
    print("[gpu-case] convergence sweep bases 32, 64, 128 f64", flush=True)
    sys.stdout.flush()
    res = bench.convergence_sweep(M, torch, bases=(32, 64, 128))
    r = res["results"]
    print(r)
    assert all(x["status"] == 0 for x in r)
    for b in r[1:]:
        assert 1.7 < b["order_u"] < 2.3, b
        assert 1.7 < b["order_S"] < 2.3, b
    # the observed order rises towards 2 as the mesh is refined
    assert r[2]["order_u"] > r[1]["order_u"] and r[2]["order_S"] > r[1]["order_S"]
    assert r[2]["eps_u"] < 3e-3 and r[2]["eps_S"] < 3e-3
