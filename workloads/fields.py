"""Analytic initial fields evaluated at caller-supplied positions (inputs only).

Positions are barycentres in coarsest-level cell units.  Every function
returns (rho, u, S) as float64 arrays with shapes (n,), (n, d), (n, d, d);
S is the symmetric strain-rate tensor in coarsest-level lattice units.
Converting S to a finer level's time unit is the consumer's job.
"""
from __future__ import annotations

import numpy as np


def tgv_fields(pos: np.ndarray, n0: int, u0: float, nu0: float = 0.0,
               t: float = 0.0, rho0: float = 1.0):
    """Two-dimensional Taylor-Green vortex on the periodic box of n0 cells
    (Sec. 4.1, Eq. tgv), rescaled to wavenumber k = 2*pi/n0.  In 3D the
    field is invariant along z.  nu0 and t (coarsest-level units) give the
    decayed state."""
    pos = np.asarray(pos, dtype=np.float64)
    n, d = pos.shape
    k = 2.0 * np.pi / n0
    x, y = pos[:, 0], pos[:, 1]
    e1 = np.exp(-2.0 * nu0 * k * k * t)
    e2 = np.exp(-4.0 * nu0 * k * k * t)
    u = np.zeros((n, d))
    u[:, 0] = -u0 * np.cos(k * x) * np.sin(k * y) * e1
    u[:, 1] = u0 * np.sin(k * x) * np.cos(k * y) * e1
    # pressure p = c_s^2 rho with c_s^2 = 1/3
    rho = rho0 - rho0 * 3.0 * (u0 * u0 / 4.0) * (np.cos(2 * k * x)
                                                  + np.cos(2 * k * y)) * e2
    S = np.zeros((n, d, d))
    sxx = u0 * k * np.sin(k * x) * np.sin(k * y) * e1
    S[:, 0, 0] = sxx
    S[:, 1, 1] = -sxx
    return rho, u, S


def fourier_perturbation(n0: int, d: int = 3, kmax: float = 4.0,
                         seed: int = 1601):
    """Divergence-free random Fourier modes with integer wavevectors
    0 < |m| <= kmax on the periodic box of n0 cells.  Complex amplitudes are
    i.i.d. standard normal, projected orthogonal to m; the field is the real
    part, so it is real by construction.  Returns (modes, amplitudes)."""
    rng = np.random.default_rng(seed)
    r = int(np.floor(kmax))
    grid = np.arange(-r, r + 1)
    ms = np.stack(np.meshgrid(*([grid] * d), indexing="ij"), -1).reshape(-1, d)
    norm2 = (ms * ms).sum(1)
    ms = ms[(norm2 > 0) & (norm2 <= kmax * kmax)]
    amp = rng.standard_normal((len(ms), d)) + 1j * rng.standard_normal((len(ms), d))
    mhat = ms / np.sqrt((ms * ms).sum(1, keepdims=True))
    amp = amp - (amp * mhat).sum(1, keepdims=True) * mhat
    return ms.astype(np.float64), amp


def _eval_modes(pos, n0, ms, amp):
    k = 2.0 * np.pi / n0
    phase = np.exp(1j * k * (pos @ ms.T))  # (n, M)
    return np.real(phase @ amp)  # (n, d)


def tgv_perturbed_fields(pos: np.ndarray, n0: int, u0: float,
                         frac: float = 0.05, kmax: float = 4.0,
                         seed: int = 1601):
    """Taylor-Green vortex plus random divergence-free Fourier modes whose
    RMS speed is ``frac`` of the Taylor-Green RMS speed (both measured on the
    cell centres of the n0^d box).  Density 1, zero strain (equilibrium)."""
    pos = np.asarray(pos, dtype=np.float64)
    n, d = pos.shape
    ms, amp = fourier_perturbation(n0, d, kmax, seed)
    c = np.arange(n0) + 0.5
    ref = np.stack(np.meshgrid(*([c] * d), indexing="ij"), -1).reshape(-1, d)
    _, u_tg_ref, _ = tgv_fields(ref, n0, u0)
    p_ref = _eval_modes(ref, n0, ms, amp)
    rms_tg = np.sqrt((u_tg_ref ** 2).sum(1).mean())
    rms_p = np.sqrt((p_ref ** 2).sum(1).mean())
    scale = frac * rms_tg / rms_p
    _, u, _ = tgv_fields(pos, n0, u0)
    u = u + scale * _eval_modes(pos, n0, ms, amp)
    return np.ones(n), u, np.zeros((n, d, d))


def uniform_fields(n: int, d: int, u, rho0: float = 1.0):
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), (n, d)).copy()
    return np.full(n, rho0), u, np.zeros((n, d, d))


def shear_wave_fields(pos: np.ndarray, z_wall: float, height: float, u0: float,
                      rho0: float = 1.0):
    """Lowest shear mode between two parallel walls: u_x = u0 sin(k (z - z_wall))
    with k = pi / height, z the last coordinate; it decays as exp(-nu k^2 t)."""
    pos = np.asarray(pos, dtype=np.float64)
    n, d = pos.shape
    k = np.pi / height
    z = pos[:, d - 1] - z_wall
    u = np.zeros((n, d))
    u[:, 0] = u0 * np.sin(k * z)
    S = np.zeros((n, d, d))
    S[:, 0, d - 1] = S[:, d - 1, 0] = 0.5 * u0 * k * np.cos(k * z)
    return np.full(n, rho0), u, S
