"""Taylor-Green vortex closed form and error norms (Sec. 4.1, Eq. tgv).

The paper's vortex lives on [0, 2 pi]^2 with u0 = 1 and t_D = 1/(2 nu).  On a
periodic box of n0 coarse cells in lattice units the same field has
wavenumber k = 2 pi / n0 and decays as exp(-2 nu k^2 t); the pressure
deviation -rho u0^2/4 (cos 2kx + cos 2ky) exp(-4 nu k^2 t) becomes a density
deviation through p = cs^2 rho.  S_xx = -S_yy = u0 k sin kx sin ky
exp(-2 nu k^2 t), S_xy = 0.  In 3D the field is taken invariant along z.
"""
from __future__ import annotations

import math

import numpy as np


def nu_from_tau(tau: float) -> float:
    """Eq. nu with dx = dt = 1: nu = (1/omega - 1/2)/3 = (tau - 1/2)/3."""
    return (tau - 0.5) / 3.0


def decay_time(n0: int, nu0: float) -> float:
    k = 2.0 * math.pi / n0
    return 1.0 / (2.0 * nu0 * k * k)


def analytic(pos, n0: int, u0: float, nu0: float, t: float, rho0: float = 1.0):
    """Velocity (n, d), density (n,), S_xx (n,) at coarse-unit positions."""
    pos = np.asarray(pos, dtype=np.float64)
    k = 2.0 * math.pi / n0
    x, y = pos[:, 0], pos[:, 1]
    g = math.exp(-2.0 * nu0 * k * k * t)
    u = np.zeros_like(pos)
    u[:, 0] = -u0 * np.cos(k * x) * np.sin(k * y) * g
    u[:, 1] = u0 * np.sin(k * x) * np.cos(k * y) * g
    p_dev = -rho0 * u0 * u0 / 4.0 * (np.cos(2 * k * x) + np.cos(2 * k * y)) * g * g
    rho = rho0 + 3.0 * p_dev
    sxx = u0 * k * np.sin(k * x) * np.sin(k * y) * g
    return u, rho, sxx


def l2_error(sim_vals, ana_vals) -> float:
    """Sec. 4.1: eps = sqrt(sum (phi_s - phi_a)^2 / sum phi_a^2), summed
    without weights over all listed values (reading taken: fluid elements of
    all levels)."""
    s = np.concatenate([np.asarray(v, dtype=np.float64).ravel() for v in sim_vals])
    a = np.concatenate([np.asarray(v, dtype=np.float64).ravel() for v in ana_vals])
    return float(np.sqrt(((s - a) ** 2).sum() / (a ** 2).sum()))


def errors(sim, n0: int, u0: float, nu0: float):
    """(eps_u, eps_Sxx) of an OracleSim at its current time, in coarsest-level
    units: u_L times (dx_L/dt_L)/(dx_L0/dt_L0) (1 under acoustic scaling,
    2^(L-L0) under diffusive), S_L times dt_L0/dt_L (2^(L-L0) acoustic,
    4^(L-L0) diffusive)."""
    us, ua, ss, sa = [], [], [], []
    for L in range(sim.L0, sim.Lmax + 1):
        t = sim.mesh.lev(L)
        pos = sim.mesh.positions(L)[:t.n_fluid]
        rho, u, S = sim.fluid_moments(L)
        u_a, _, sxx_a = analytic(pos, n0, u0, nu0, float(sim.time))
        us.append(u.detach().numpy()[0] * sim.unit_ratio(L))
        ua.append(u_a[:, 0])
        ss.append(S.detach().numpy()[0, 0] * float(sim.n_sub) ** (L - sim.L0))
        sa.append(sxx_a)
    return l2_error(us, ua), l2_error(ss, sa)
