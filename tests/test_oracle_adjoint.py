"""Pins of the oracle's reverse pass against central finite differences of
the forward oracle and against exact complex-step tangents of it (both
independent of automatic differentiation)."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, mesh


def _fields(m, n0, fn):
    rho, u, S = {}, {}, {}
    for L in range(m.level0, m.lmax + 1):
        t = m.lev(L)
        pos = m.positions(L)[:t.n_fluid]
        r, uu, SS = fn(pos)
        rho[L], u[L], S[L] = r, uu, SS * 2.0 ** -(L - m.level0)
    return rho, u, S


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19"])
def test_ke_gradient_matches_central_differences(stencil):
    spec = (W.refined_box_mesh("D3Q19", 3, 2, 6) if stencil == "D3Q19"
            else W.refined_box_mesh("D2Q9", 4, 4, 12))
    m = mesh.build(spec)
    n0 = spec.box_extent[0]
    rho, u, S = _fields(m, n0, lambda p: W.tgv_perturbed_fields(p, n0, 0.03))
    J, g_tau, g_u, _ = adjoint.gradient(m, 0.57, rho, u, S, 4)
    rng = np.random.default_rng(1)
    for _ in range(2):
        du = {L: rng.normal(size=u[L].shape) for L in u}
        fd = adjoint.central_difference(m, 0.57, rho, u, S, 4, du=du, eps=1e-5)
        ad = sum((g_u[L] * du[L]).sum() for L in u)
        assert abs(fd - ad) <= 1e-7 * abs(ad)
    # single components on both levels
    for L in u:
        du = {K: np.zeros_like(u[K]) for K in u}
        du[L][3, 0] = 1.0
        fd = adjoint.central_difference(m, 0.57, rho, u, S, 4, du=du, eps=1e-5)
        assert abs(fd - g_u[L][3, 0]) <= 1e-7 * max(abs(fd), 1e-6)
    fd = adjoint.central_difference(m, 0.57, rho, u, S, 4, dtau=1.0, eps=1e-6)
    assert abs(fd - g_tau) <= 1e-7 * abs(g_tau)


def _compact_sphere():
    return W.sphere_channel_mesh(8, 2, l0_per_d=4, length=(-1.5, 2.0), half_width=1.5,
                                 boxes_in_d=((-0.75, 1.0, 0.75),))


@pytest.mark.parametrize("objective,steps", [("ke", 3), ("drag_x", 6)])
def test_gradient_wrt_inflow_and_tau(objective, steps):
    """Compact sphere channel: both objectives feel the inflow face within
    the run, so d/du_in is far from zero and is checked, as is d/dtau0."""
    m = mesh.build(_compact_sphere())
    uin = np.array([0.04, 0.0, 0.0])
    rho, u, S = {}, {}, {}
    for L in range(m.level0, m.lmax + 1):
        rho[L], u[L], S[L] = W.uniform_fields(m.lev(L).n_fluid, 3, uin)
    J, g_tau, g_u, g_in = adjoint.gradient(m, 0.6, rho, u, S, steps,
                                           objective=objective, u_in=uin)
    assert J > 0 and abs(g_in[0]) > 1.0
    fd = adjoint.central_difference(m, 0.6, rho, u, S, steps, objective=objective,
                                    duin=np.array([1.0, 0, 0]), u_in=uin, eps=1e-6)
    assert abs(fd - g_in[0]) <= 1e-6 * abs(fd)
    fd = adjoint.central_difference(m, 0.6, rho, u, S, steps, objective=objective,
                                    dtau=1.0, u_in=uin, eps=1e-6)
    assert abs(fd - g_tau) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("objective,steps", [("ke", 3), ("drag_x", 6)])
def test_gradient_with_curved_walls(objective, steps):
    """The reverse pass through the linear interpolated bounce-back (Sec.
    2.3) on the sphere's links, against central differences of the forward
    run (d/du_in, d/dtau0 and a random initial-velocity direction)."""
    spec = _compact_sphere()
    m = mesh.build(spec)
    walls = W.sphere_wall_links(spec, m.lattice.c)
    uin = np.array([0.04, 0.0, 0.0])
    rho, u, S = {}, {}, {}
    for L in range(m.level0, m.lmax + 1):
        rho[L], u[L], S[L] = W.uniform_fields(m.lev(L).n_fluid, 3, uin)
    J, g_tau, g_u, g_in = adjoint.gradient(m, 0.6, rho, u, S, steps, objective=objective,
                                           u_in=uin, walls=walls)
    assert J > 0 and abs(g_in[0]) > 1.0
    fd = adjoint.central_difference(m, 0.6, rho, u, S, steps, objective=objective,
                                    duin=np.array([1.0, 0, 0]), u_in=uin, eps=1e-6,
                                    walls=walls)
    assert abs(fd - g_in[0]) <= 1e-6 * abs(fd)
    fd = adjoint.central_difference(m, 0.6, rho, u, S, steps, objective=objective,
                                    dtau=1.0, u_in=uin, eps=1e-6, walls=walls)
    assert abs(fd - g_tau) <= 1e-6 * abs(fd)
    rng = np.random.default_rng(7)
    du = {L: rng.normal(size=u[L].shape) for L in u}
    fd = adjoint.central_difference(m, 0.6, rho, u, S, steps, objective=objective,
                                    du=du, u_in=uin, eps=1e-6, walls=walls)
    ad = sum(float((g_u[L] * du[L]).sum()) for L in u)
    assert abs(fd - ad) <= 1e-6 * abs(fd) + 1e-12
    # the walls change the gradient
    _, _, _, g_in_h = adjoint.gradient(m, 0.6, rho, u, S, steps, objective=objective, u_in=uin)
    assert abs(g_in_h[0] - g_in[0]) > 1e-4 * abs(g_in[0])


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19"])
def test_reverse_pass_equals_complex_step_tangents(stencil):
    """Dot-product test with exact tangents: the forward oracle run in
    complex128 with the input perturbed by i h d (h = 1e-30) gives
    dJ/dx . d as Im J / h with no cancellation, so the reverse pass must
    match it to rounding (1e-12), along a random initial-velocity
    direction and along tau0."""
    import torch
    from oracle.solver import OracleSim
    spec = (W.refined_box_mesh("D3Q19", 3, 2, 6) if stencil == "D3Q19"
            else W.refined_box_mesh("D2Q9", 4, 4, 12))
    m = mesh.build(spec)
    n0 = spec.box_extent[0]
    rho, u, S = _fields(m, n0, lambda p: W.tgv_perturbed_fields(p, n0, 0.03))
    J, g_tau, g_u, _ = adjoint.gradient(m, 0.57, rho, u, S, 4)
    rng = np.random.default_rng(7)
    du = {L: rng.normal(size=u[L].shape) for L in u}
    h = 1e-30

    def tangent(tau, uu):
        sim = OracleSim(m, torch.tensor(tau, dtype=torch.complex128), poison=False,
                        dtype=torch.complex128)
        sim.init(rho, uu, S)
        sim.step(4)
        Jc = sim.kinetic_energy()
        assert abs(float(Jc.real) - J) <= 1e-14 * abs(J)
        return float(Jc.imag) / h

    ad = sum((g_u[L] * du[L]).sum() for L in u)
    cs = tangent(0.57, {L: np.asarray(u[L]) + 1j * h * du[L] for L in u})
    assert abs(cs - ad) <= 1e-12 * abs(ad), (cs, ad)
    cs = tangent(0.57 + 1j * h, u)
    assert abs(cs - g_tau) <= 1e-12 * abs(g_tau), (cs, g_tau)


def test_inflow_gradient_equals_complex_step_tangent():
    """The drag's derivative with respect to the free-stream velocity (EQ
    faces and momentum exchange on the sphere) against its complex-step
    tangent, to rounding."""
    import torch
    from oracle.solver import OracleSim
    m = mesh.build(_compact_sphere())
    uin = np.array([0.04, 0.0, 0.0])
    rho, u, S = {}, {}, {}
    for L in range(m.level0, m.lmax + 1):
        rho[L], u[L], S[L] = W.uniform_fields(m.lev(L).n_fluid, 3, uin)
    _, _, _, g_in = adjoint.gradient(m, 0.6, rho, u, S, 6, objective="drag_x", u_in=uin)
    h = 1e-30
    sim = OracleSim(m, torch.tensor(0.6, dtype=torch.complex128),
                    u_in=torch.tensor(uin + 1j * h * np.array([1.0, 0.0, 0.0]),
                                      dtype=torch.complex128),
                    poison=False, dtype=torch.complex128)
    sim.init(rho, u, S)
    sim.step(6)
    cs = float(sim.force()[0].imag) / h
    assert abs(cs - g_in[0]) <= 1e-12 * abs(g_in[0]), (cs, g_in[0])
