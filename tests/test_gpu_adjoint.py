"""GPU adjoint of the multilevel step against (a) the oracle's reverse pass
(automatic differentiation of the FP64 oracle run) and (b) central finite
differences of the library's own FP64 forward.

Tolerances: F64 gradients agree with the oracle to 1e-8 relative (max
norm); F32 to 2e-4 (single-precision forward and reverse arithmetic over a
few steps of O(1) pdfs).
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as oadj
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


def gpu_gradient(spec, precision, tau0, fields, steps, objective="ke", u_in=None, walls=False):
    import paper_1601_06984_amd as M
    plan = None
    if walls:   # a function of the velocity set giving the wall links
        plan = M.Plan.from_spec(spec)
        plan.set_walls(*walls(M.lattice(spec.stencil)[0]))
    sim = H.gpu_sim(spec, precision, tau0, fields, u_in=u_in, plan=plan)
    sim.adjoint_attach()
    ckpts = []
    for _ in range(steps):
        ckpts.append(sim.save_checkpoint())
        sim.step(1)
    mask = M.DIAG_KE if objective == "ke" else M.DIAG_FORCE
    J = float(sim.diagnostics(mask)[0])
    sim.adjoint_seed(objective)
    for t in reversed(range(steps)):
        sim.adjoint_step(ckpts[t])
    n = sim.plan.n_levels
    rho = [sim.inputs[k][0] for k in range(n)]
    u = [sim.inputs[k][1] for k in range(n)]
    S = [sim.inputs[k][2] for k in range(n)]
    du = sim.adjoint_init(rho, u, S)
    dtau, domega, duin = sim.adjoint_params()
    return sim, J, [d.cpu().numpy() for d in du], dtau, duin


def oracle_gradient(spec, tau0, fields, steps, objective="ke", u_in=None, walls=False):
    om = omesh.build(spec)
    wl = walls(om.lattice.c) if walls else None
    rho, u, S = {}, {}, {}
    for L in range(om.level0, om.lmax + 1):
        pos = om.positions(L)[:om.lev(L).n_fluid]
        r, uu, SS = fields(pos)
        rho[L], u[L], S[L] = r, uu, SS * 2.0 ** -(L - om.level0)
    J, gt, gu, gin = oadj.gradient(om, tau0, rho, u, S, steps, objective, u_in=u_in, walls=wl)
    return om, J, gt, gu, gin


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _compare(sim, om, du_gpu, gu_or):
    worst = 0.0
    for k in range(sim.plan.n_levels):
        L = sim.plan.level0 + k
        g2o = H.gpu_to_oracle(sim.plan, om, k)
        nf = sim.plan.info[k]["n_fluid"]
        want = gu_or[L][g2o[:nf]].T          # (d, n_fluid) in GPU order
        worst = max(worst, _rel(du_gpu[k], want))
    return worst


CASES = [
    ("d3q19_2lev_ke", lambda: W.refined_box_mesh("D3Q19", 4, 4, 12), 16, 4, 0.56),
    ("d2q9_2lev_ke", lambda: W.refined_box_mesh("D2Q9", 5, 8, 24), 32, 6, 0.6),
    ("d2q9_3lev_ke", lambda: W.refined_box_mesh("D2Q9", 5, 8, 24, extra_levels=[(20, 44)]), 32, 3, 0.7),
    # a coarse level whose blocks hold Morton directions of the pull table
    ("d3q19_morton_ke", lambda: W.refined_box_mesh("D3Q19", 5, 14, 18), 32, 3, 0.56),
    ("d3q27_2lev_ke", lambda: W.refined_box_mesh("D3Q27", 4, 4, 12), 16, 4, 0.56),
    ("d3q27_morton_ke", lambda: W.refined_box_mesh("D3Q27", 5, 14, 18), 32, 3, 0.56),
]


@pytest.mark.parametrize("name,spec_fn,n0,steps,tau0", CASES)
@pytest.mark.parametrize("precision,tol", [("f64", 1e-8), ("f32", 2e-4)])
def test_ke_gradient_matches_oracle_reverse(name, spec_fn, n0, steps, tau0, precision, tol, morton):
    spec = spec_fn()
    fields = lambda p: W.tgv_perturbed_fields(p, n0, 0.03)
    _say(name, precision, steps)
    sim, J, du, dtau, _ = gpu_gradient(spec, precision, tau0, fields, steps)
    om, Jo, gto, guo, _ = oracle_gradient(spec, tau0, fields, steps)
    assert abs(J - Jo) <= 1e-6 * abs(Jo)
    err = _compare(sim, om, du, guo)
    print("du rel err", err, "dtau", dtau, gto)
    assert err < tol
    assert abs(dtau - gto) <= tol * abs(gto)


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19"])
def test_grouped_reverse_launches_match_per_level(stencil):
    """The reverse step launches consecutive reverse stream-collides of
    different levels (and the tape's forward kernels) together; a profiled
    run launches one level at a time.  Both give the same bits."""
    if stencil == "D3Q19":
        spec = W.refined_box_mesh("D3Q19", 4, 2, 14, extra_levels=[(10, 18)])
        n0 = 16
    else:
        spec = W.refined_box_mesh("D2Q9", 5, 8, 24, extra_levels=[(20, 44)])
        n0 = 32
    fields = lambda p: W.tgv_perturbed_fields(p, n0, 0.03)
    _say("grouped vs per-level reverse", stencil)
    out = []
    for prof in (False, True):
        sim = H.gpu_sim(spec, "f64", 0.7, fields)
        sim.adjoint_attach()
        if prof:
            sim.profile(True)
        ckpts = []
        for _ in range(3):
            ckpts.append(sim.save_checkpoint())
            sim.step(1)
        sim.adjoint_seed("ke")
        for t in reversed(range(3)):
            sim.adjoint_step(ckpts[t])
        lam = [sim.adjoint_lambda(k).clone() for k in range(sim.plan.n_levels)]
        dtau, _, duin = sim.adjoint_params()
        out.append((lam, dtau))
    for a, b in zip(out[0][0], out[1][0]):
        assert torch.equal(a, b)
    assert out[0][1] == out[1][1]


def _compact_sphere(stencil="D3Q19"):
    return W.sphere_channel_mesh(8, 2, l0_per_d=4, length=(-1.5, 2.0), half_width=1.5,
                                 boxes_in_d=((-0.75, 1.0, 0.75),), stencil=stencil)


@pytest.mark.parametrize("stencil", ["D3Q19", "D3Q27"])
@pytest.mark.parametrize("objective,steps", [("ke", 3), ("drag_x", 6)])
@pytest.mark.parametrize("precision,tol", [("f64", 1e-8), ("f32", 5e-4)])
def test_gradients_with_boundaries(objective, steps, precision, tol, stencil):
    """Bounce-back, equilibrium faces (d/du_in, far from zero here) and the
    copy outlet in reverse, against the oracle's reverse pass."""
    spec = _compact_sphere(stencil)
    uin = np.array([0.04, 0.0, 0.0])
    fields = lambda p: W.uniform_fields(len(p), 3, uin)
    _say("sphere", objective, precision)
    sim, J, du, dtau, duin = gpu_gradient(spec, precision, 0.6, fields, steps, objective, u_in=uin)
    om, Jo, gto, guo, gino = oracle_gradient(spec, 0.6, fields, steps, objective, u_in=uin)
    assert abs(J - Jo) <= 1e-5 * abs(Jo)
    print("duin", duin, gino, "dtau", dtau, gto)
    assert abs(gino[0]) > 1.0
    assert np.abs(duin - gino).max() <= tol * np.abs(gino).max()
    assert abs(dtau - gto) <= tol * abs(gto)
    assert _compare(sim, om, du, guo) < tol * 10


@pytest.mark.parametrize("stencil", ["D3Q19", "D3Q27"])
@pytest.mark.parametrize("objective,steps", [("ke", 3), ("drag_x", 6)])
@pytest.mark.parametrize("precision,tol", [("f64", 1e-8), ("f32", 5e-4)])
def test_gradients_with_curved_walls(objective, steps, precision, tol, stencil):
    """The sphere's links with wall fractions (linear interpolated
    bounce-back) in reverse: the transposed wall pre-pass and the drag seed
    of the interpolated returning values, against the oracle's reverse pass."""
    spec = _compact_sphere(stencil)
    uin = np.array([0.04, 0.0, 0.0])
    fields = lambda p: W.uniform_fields(len(p), 3, uin)
    _say("sphere walls", objective, precision, stencil)
    links = lambda c: W.sphere_wall_links(spec, c)
    sim, J, du, dtau, duin = gpu_gradient(spec, precision, 0.6, fields, steps, objective,
                                          u_in=uin, walls=links)
    om, Jo, gto, guo, gino = oracle_gradient(spec, 0.6, fields, steps, objective, u_in=uin,
                                             walls=links)
    assert abs(J - Jo) <= 1e-5 * abs(Jo)
    print("duin", duin, gino, "dtau", dtau, gto)
    assert abs(gino[0]) > 1.0
    assert np.abs(duin - gino).max() <= tol * np.abs(gino).max()
    assert abs(dtau - gto) <= tol * abs(gto)
    assert _compare(sim, om, du, guo) < tol * 10


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("q_low,q_high", [(0.7, 0.8), (0.3, 0.6)])
@pytest.mark.parametrize("height", [3, 4])
def test_gradients_with_walls_on_both_sides_of_a_row(stencil, q_low, q_high, height):
    """One or two fluid rows between two walls: one link's value reads the
    entry the opposite link's value replaces (one row), or two links' terms
    meet in one entry of the other row (two rows); F64 gradient of the
    kinetic energy against the oracle's reverse pass."""
    spec = W.plane_channel_mesh(stencil, 5, 4, height)
    d = spec.dim
    links = lambda c: W.plane_wall_links(spec, c, q_low, q_high)
    fields = lambda p: W.tgv_perturbed_fields(p, 4, 0.03)
    _say("two rows between walls", stencil, q_low, q_high)
    sim, J, du, dtau, _ = gpu_gradient(spec, "f64", 0.8, fields, 4, walls=links)
    om, Jo, gto, guo, _ = oracle_gradient(spec, 0.8, fields, 4, walls=links)
    assert abs(J - Jo) <= 1e-10 * abs(Jo)
    assert _compare(sim, om, du, guo) < 1e-8
    assert abs(dtau - gto) <= 1e-8 * abs(gto)


def test_f64_adjoint_matches_central_differences_of_gpu_forward():
    """Directional derivative along a random initial-velocity perturbation:
    the GPU adjoint against (J(u + e d) - J(u - e d)) / 2e of the GPU FP64
    forward itself, e = 1e-4 as in the adjoint configuration."""
    import paper_1601_06984_amd as M
    spec = W.refined_box_mesh("D3Q19", 4, 4, 12)
    base = lambda p: W.tgv_perturbed_fields(p, 16, 0.02)
    steps = 6
    _say("fd check f64")
    sim, J, du, dtau, _ = gpu_gradient(spec, "f64", 0.55, base, steps)
    rng = np.random.default_rng(3)
    plan = sim.plan
    dirs = {}
    for k in range(plan.n_levels):
        dirs[k] = rng.normal(size=(plan.d, plan.info[k]["n_fluid"]))
    ad = sum(float((du[k] * dirs[k]).sum()) for k in dirs)

    def J_of(eps):
        s2 = M.Sim(plan, "f64", 0.55)
        for k in range(plan.n_levels):
            r, u, S = sim.inputs[k]
            s2.init(k, r, (u + eps * torch.tensor(dirs[k], device=u.device)).contiguous(), S)
        s2.fill_ghosts()
        s2.step(steps)
        return float(s2.diagnostics(M.DIAG_KE)[0])
    eps = 1e-4
    fd = (J_of(eps) - J_of(-eps)) / (2 * eps)
    print("fd", fd, "adjoint", ad)
    assert abs(fd - ad) <= 1e-6 * abs(ad)


F16S_CASES = [
    ("d3q19_2lev_ke", lambda: W.refined_box_mesh("D3Q19", 4, 4, 12), "ke", 4, 0.56, None),
    ("sphere_ke", _compact_sphere, "ke", 3, 0.6, [0.04, 0.0, 0.0]),
    ("sphere_drag_x", _compact_sphere, "drag_x", 6, 0.6, [0.04, 0.0, 0.0]),
]


@pytest.mark.parametrize("name,spec_fn,objective,steps,tau0,uin", F16S_CASES)
def test_f16s_gradient_matches_oracle_reverse(name, spec_fn, objective, steps, tau0, uin):
    """FP16-shift storage.  The reverse pass treats the storage rounding as
    the identity: it is the FP32 adjoint taken along the rounded forward
    trajectory.  Each stored deviation g = f - w rho0 keeps 11 significant
    bits (relative rounding 2^-11 = 4.9e-4 per store), so the forward state
    and with it every linearisation point differ from the FP64 oracle's by
    a few 1e-4 of the deviations after a few steps; the gradients follow
    at that order.  Bound: 5e-3 relative (max norm) for dJ/du0, dJ/dtau0
    and dJ/du_in, against the oracle's reverse pass; J within 1e-3."""
    spec = spec_fn()
    if uin is None:
        fields = lambda p: W.tgv_perturbed_fields(p, 16, 0.03)
        u_in = None
    else:
        u_in = np.array(uin)
        fields = lambda p: W.uniform_fields(len(p), 3, u_in)
    _say("f16s adjoint", name)
    sim, J, du, dtau, duin = gpu_gradient(spec, "f16s", tau0, fields, steps, objective,
                                          u_in=u_in)
    om, Jo, gto, guo, gino = oracle_gradient(spec, tau0, fields, steps, objective, u_in=u_in)
    err_u = _compare(sim, om, du, guo)
    err_t = abs(dtau - gto) / abs(gto)
    print(name, "J", J, Jo, "du rel", err_u, "dtau rel", err_t, "duin", duin, gino)
    assert abs(J - Jo) <= 1e-3 * abs(Jo)
    assert err_u < 5e-3
    assert err_t < 5e-3
    if u_in is not None:
        assert np.abs(duin - gino).max() <= 5e-3 * np.abs(gino).max()
