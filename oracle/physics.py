"""Moments, equilibrium, strain rate and BGK collision (Sec. 2.1).

All functions act on pdf tensors of shape (q, N) and work for real or
complex float64 tensors and under autograd.

Reading taken for Eq. feq: the printed '+ u.u/(2 cs^2)' is a sign garble;
the second-order truncation of the Maxwellian has '- u.u/(2 cs^2)', which is
the only sign for which sum_i f_i^eq = rho.

Reading taken for the initial non-equilibrium part (Sec. 4.1): the printed
prefactor is dimensionally garbled; the first-order Chapman-Enskog form
f_i^neq = -(w_i rho / (cs^2 omega)) Q_i : S with Q_i = c_i c_i - cs^2 I is
used, which the strain-rate formula of Sec. 2.1 maps back to S exactly.
"""
from __future__ import annotations

import torch

from .lattice import CS2, Lattice


def level_tau(tau0, level: int, level0: int):
    """Eq. fneq_scale applied once per level jump with m = 2:
    1/omega_f - 1/2 = 2 (1/omega_c - 1/2), i.e. tau_L = 1/2 + 2^(L-L0)(tau0-1/2)."""
    return 0.5 + (2 ** (level - level0)) * (tau0 - 0.5)


def moments(f: torch.Tensor, lat: Lattice):
    """Eq. (rho, rho u): rho = sum_i f_i, rho u = sum_i c_i f_i."""
    c = lat.c_t(f.real.dtype).to(f.dtype)
    rho = f.sum(0)
    j = c.t() @ f                      # (d, N)
    return rho, j / rho


def equilibrium(rho: torch.Tensor, u: torch.Tensor, lat: Lattice) -> torch.Tensor:
    """Eq. feq with the sign reading above:
    f_i^eq = w_i rho (1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2))."""
    c = lat.c_t().to(u.dtype)
    w = lat.w_t().to(u.dtype)
    cu = c @ u                          # (q, N)
    uu = (u * u).sum(0)                 # (N,)
    return w[:, None] * rho[None, :] * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2)
                                        - uu[None, :] / (2.0 * CS2))


def second_moment(g: torch.Tensor, lat: Lattice) -> torch.Tensor:
    """sum_i c_ia c_ib g_i -> (d, d, N)."""
    c = lat.c_t().to(g.dtype)
    return torch.einsum("ia,ib,in->abn", c, c, g)


def strain_rate(f: torch.Tensor, omega, lat: Lattice):
    """Sec. 2.1: S_ab = -(3 omega / (2 rho)) sum_i c_ia c_ib f_i^neq with
    f^neq = f - f^eq(rho, u) of the same pdfs.  Returns (rho, u, S, fneq)."""
    rho, u = moments(f, lat)
    fneq = f - equilibrium(rho, u, lat)
    S = -(3.0 * omega / (2.0 * rho))[None, None, :] * second_moment(fneq, lat)
    return rho, u, S, fneq


def fneq_from_strain(rho: torch.Tensor, S: torch.Tensor, omega, lat: Lattice) -> torch.Tensor:
    """f_i^neq = -(w_i rho / (cs2 omega)) Q_i : S, Q_i = c_i c_i - cs2 I."""
    c = lat.c_t().to(S.dtype)
    w = lat.w_t().to(S.dtype)
    eye = torch.eye(lat.d, dtype=S.dtype)
    Q = c[:, :, None] * c[:, None, :] - CS2 * eye[None]          # (q, d, d)
    QS = torch.einsum("iab,abn->in", Q, S)
    return -(w[:, None] * rho[None, :] / (CS2 * omega)) * QS


def collide(f: torch.Tensor, omega, lat: Lattice) -> torch.Tensor:
    """Eq. bgk right-hand side: f* = f - omega (f - f^eq)."""
    rho, u = moments(f, lat)
    return f - omega * (f - equilibrium(rho, u, lat))
