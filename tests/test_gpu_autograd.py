"""torch.autograd front end with K-step checkpointing."""
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


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1601_06984_amd  # noqa: F401


def _inputs(plan, fields, dev):
    rho, u, S = [], [], []
    for k in range(plan.n_levels):
        nf = plan.info[k]["n_fluid"]
        pos = H.level_positions_from_coords(plan.export(k, "coords")[:, :nf], plan.level0 + k,
                                            plan.level0)
        r, uu, SS = fields(pos)
        SS = SS * 2.0 ** -k
        rho.append(torch.tensor(r, device=dev))
        u.append(torch.tensor(np.ascontiguousarray(uu.T), device=dev))
        S.append(torch.tensor(np.ascontiguousarray(H.strain_components(SS, plan.d)), device=dev))
    return rho, u, S


def _run(plan, precision, rho, u, S, tau0, n, K, objective="ke", u_in=None, snapshots=None):
    from paper_1601_06984_amd import autograd as AG
    u0 = [x.clone().requires_grad_(True) for x in u]
    tau = torch.tensor(tau0, dtype=torch.float64, requires_grad=True)
    uin = None if u_in is None else torch.tensor(u_in, dtype=torch.float64, requires_grad=True)
    J = AG.objective(plan, rho, u0, tau, n, S=S, u_in=uin, precision=precision,
                     checkpoint_every=K, objective=objective, max_snapshots=snapshots)
    J.backward()
    return float(J), [x.grad.clone() for x in u0], float(tau.grad), \
        (uin.grad.clone() if uin is not None else None)


def test_checkpointed_gradient_equals_stepwise_adjoint_and_oracle():
    import paper_1601_06984_amd as M
    from tests.test_gpu_adjoint import _compare, gpu_gradient, oracle_gradient
    spec = W.refined_box_mesh("D3Q19", 4, 4, 12)
    fields = lambda p: W.tgv_perturbed_fields(p, 16, 0.03)
    plan = M.Plan.from_spec(spec)
    rho, u, S = _inputs(plan, fields, "cuda")
    _say("autograd K=3 n=7 f64")
    J, gu, gt, _ = _run(plan, "f64", rho, u, S, 0.56, 7, 3)
    sim, J2, du, dtau, _ = gpu_gradient(spec, "f64", 0.56, fields, 7)
    assert J == J2
    for k in range(plan.n_levels):
        assert torch.equal(gu[k].cpu(), torch.tensor(du[k]))
    assert gt == dtau
    om, Jo, gto, guo, _ = oracle_gradient(spec, 0.56, fields, 7)
    assert _compare(sim, om, [g.cpu().numpy() for g in gu], guo) < 1e-8
    assert abs(gt - gto) < 1e-8 * abs(gto)


def test_bisection_checkpointing_matches_stored_states():
    """Reversing a segment by recursive bisection with few stored states
    recomputes the same forward states, so the gradient is bitwise the one
    obtained by keeping every step state; so does the budget taken from the
    free device memory."""
    import paper_1601_06984_amd as M
    spec = W.refined_box_mesh("D3Q19", 4, 4, 12)
    fields = lambda p: W.tgv_perturbed_fields(p, 16, 0.03)
    plan = M.Plan.from_spec(spec)
    rho, u, S = _inputs(plan, fields, "cuda")
    _say("autograd snapshots None/2/0/auto, 11 steps, K=11 and K=4, f32")
    ref = _run(plan, "f32", rho, u, S, 0.56, 11, 11)
    for K, snaps in ((11, 2), (11, 0), (4, 1), (11, "auto")):
        J, gu, gt, _ = _run(plan, "f32", rho, u, S, 0.56, 11, K, snapshots=snaps)
        assert J == ref[0] and gt == ref[2]
        for a, b in zip(gu, ref[1]):
            assert torch.equal(a, b)


def test_drag_gradient_wrt_inflow_through_autograd():
    import paper_1601_06984_amd as M
    from tests.test_gpu_adjoint import gpu_gradient
    spec = W.sphere_channel_mesh(8, 2, l0_per_d=4, length=(-1.5, 2.0), half_width=1.5,
                                 boxes_in_d=((-0.75, 1.0, 0.75),))
    uin = [0.04, 0.0, 0.0]
    fields = lambda p: W.uniform_fields(len(p), 3, uin)
    plan = M.Plan.from_spec(spec)
    rho, u, S = _inputs(plan, fields, "cuda")
    _say("autograd drag u_in f64")
    J, gu, gt, gin = _run(plan, "f64", rho, u, S, 0.6, 7, 3, objective="drag_x", u_in=uin)
    _, J2, du, dtau, duin = gpu_gradient(spec, "f64", 0.6, fields, 7, "drag_x", u_in=np.array(uin))
    assert J == J2 and gt == dtau
    assert abs(float(gin[0])) > 1.0
    assert np.array_equal(gin.numpy(), duin)


@pytest.mark.timeout(600)
def test_adjoint_configuration_central_differences():
    """The adjoint workload at full size: D3Q19 64^3 coarse with the central
    32^3 refined, Taylor-Green (u0 = 0.02, Re = 100) plus 5% random
    divergence-free Fourier modes |k| <= 4 (seed 1601), kinetic energy
    after 200 coarse steps, checkpoints every 20 steps, FP32 adjoint.
    Checked against central differences (eps = 1e-4) of the FP64 forward
    along 8 random directions, 8 single components and tau0."""
    import paper_1601_06984_amd as M
    spec = W.refined_box_mesh("D3Q19", 6, 16, 48)
    n0, u0 = 64, 0.02
    tau0 = 0.5 + 3 * u0 * n0 / (2 * np.pi * 100)
    fields = lambda p: W.tgv_perturbed_fields(p, n0, u0, frac=0.05, kmax=4.0, seed=1601)
    plan = M.Plan.from_spec(spec)
    rho, u, S = _inputs(plan, fields, "cuda")
    steps, K = 200, 20
    _say("adjoint config f32 200 steps K=20")
    J, gu32, gt32, _ = _run(plan, "f32", rho, u, S, tau0, steps, K)
    _say("adjoint config f64 200 steps K=20")
    J64, gu64, gt64, _ = _run(plan, "f64", rho, u, S, tau0, steps, K)

    def J_of(du=None, dtau=0.0):
        s2 = M.Sim(plan, "f64", tau0 + dtau)
        for k in range(plan.n_levels):
            uu = u[k] if du is None else (u[k] + du[k]).contiguous()
            s2.init(k, rho[k], uu, S[k])
        s2.fill_ghosts()
        s2.step(steps)
        return float(s2.diagnostics(M.DIAG_KE)[0])

    eps = 1e-4
    rng = np.random.default_rng(1601)
    rows = []
    for t in range(16):
        if t < 8:
            d = [torch.tensor(rng.normal(size=tuple(x.shape)), device="cuda") for x in u]
        else:
            d = [torch.zeros_like(x) for x in u]
            k = t % plan.n_levels
            j = int(rng.integers(plan.info[k]["n_fluid"]))
            d[k][t % plan.d, j] = 1.0
        fd = (J_of([eps * x for x in d]) - J_of([-eps * x for x in d])) / (2 * eps)
        a32 = sum(float((g * x).sum()) for g, x in zip(gu32, d))
        a64 = sum(float((g * x).sum()) for g, x in zip(gu64, d))
        rows.append((fd, a32, a64))
    fd_tau = (J_of(dtau=eps) - J_of(dtau=-eps)) / (2 * eps)
    print("J", J, J64)
    for r in rows:
        print("dir fd %.6e  f32 %.6e  f64 %.6e" % r)
    print("tau fd %.6e f32 %.6e f64 %.6e" % (fd_tau, gt32, gt64))
    scale = max(abs(r[0]) for r in rows)
    for fd, a32, a64 in rows:
        assert abs(a64 - fd) <= 1e-5 * max(abs(fd), 1e-3 * scale)
        assert abs(a32 - fd) <= 2e-3 * max(abs(fd), 1e-2 * scale)
    # tau0 sits 0.006 above 1/2: the O(eps^2) term of the central difference
    # is ~(eps / (tau0 - 1/2))^2 ~ 3e-4 relative
    assert abs(gt64 - fd_tau) <= 1e-3 * abs(fd_tau)
    assert abs(gt32 - fd_tau) <= 3e-3 * abs(fd_tau)
