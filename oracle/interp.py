"""Four-source compact interpolation (Sec. 2.2).

3D: the quadratic velocity polynomial with 30 coefficients, fixed by the
12 velocity equations at the four sources (Eq. compact_3D_u) and the 18
equations that equate the derivatives of the polynomial's strain rate to
finite differences of the sources' strain rates (Eq. compact_3D_s).  The
30x30 system is assembled as printed (basis 1, x, y, z, x^2, y^2, z^2, xy,
yz, xz per velocity component) and solved with LAPACK.  The finite
difference of Eq. compact_3D_s is the gradient of the affine function
through the four sources' values, which is exactly the printed formula for
the tetrahedron H(0,0,0), K(1,1,0), M(1,0,1), N(0,1,1) and its mirror
images.

2D (reading taken; the paper defers the 2D algorithm to Geier's work): the
six quadratic coefficients come from the six derivatives of S_xx, S_yy,
S_xy, each taken as the gradient of the bilinear interpolant of the four
source values at the square's centre; the remaining part of the velocity is
the bilinear interpolant of the residuals u_k - Q(x_k).  Both 2D and 3D are
exact for quadratic velocity fields with linear strain rates.

Density (pressure) and f^neq are interpolated linearly: barycentric weights
on the tetrahedron in 3D, bilinear weights on the square in 2D.

Steps 1-5 of Sec. 2.2 are in :func:`fill`.  Reading taken for Step 4: omega
is read as a relaxation rate per unit physical time, so
f^neq_target = f^neq * (omega_s / omega_t) * (dt_t / dt_s).
"""
from __future__ import annotations

import torch

from . import physics

_BASIS3 = ("1", "x", "y", "z", "xx", "yy", "zz", "xy", "yz", "xz")


def _basis3(p):
    x, y, z = (float(v) for v in p)
    return [1.0, x, y, z, x * x, y * y, z * z, x * y, y * z, x * z]


def _hess3(j):
    """Second-derivative matrix (constant) of basis function j."""
    H = [[0.0] * 3 for _ in range(3)]
    name = _BASIS3[j]
    if len(name) == 2:
        a, b = ("xyz".index(name[0]), "xyz".index(name[1]))
        if a == b:
            H[a][a] = 2.0
        else:
            H[a][b] = H[b][a] = 1.0
    return H


def affine_gradient_matrix(pos, dtype=torch.float64):
    """G (3, 4) with grad = G @ values for the affine function through the
    four points ``pos`` (4, 3)."""
    A = torch.tensor([[1.0] + [float(v) for v in p] for p in pos], dtype=dtype)
    return torch.linalg.inv(A)[1:, :]


_STRAIN_ORDER = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2))


def compact3d_system(pos, dtype=torch.float64):
    """The 30x30 matrix: rows 0..11 Eq. compact_3D_u (source k, component m),
    rows 12..29 Eq. compact_3D_s (component ab in the printed order, then
    derivative direction x, y, z); unknown m*10+j is the coefficient of basis
    function j in velocity component m."""
    M = torch.zeros((30, 30), dtype=dtype)
    r = 0
    for p in pos:
        b = _basis3(p)
        for m in range(3):
            for j in range(10):
                M[r, m * 10 + j] = b[j]
            r += 1
    for (a, bb) in _STRAIN_ORDER:
        for g in range(3):
            # d/dg S_ab = 1/2 (d_g d_a u_b + d_g d_b u_a)
            for j in range(10):
                H = _hess3(j)
                M[r, bb * 10 + j] += 0.5 * H[g][a]
                M[r, a * 10 + j] += 0.5 * H[g][bb]
            r += 1
    return M


def compact3d(pos, target, u_src, S_src):
    """Quadratic compact interpolation in 3D.

    pos (4, 3) source coordinates, target (3,), u_src (n, 4, 3),
    S_src (n, 4, 3, 3) -> u (n, 3)."""
    dtype = u_src.dtype
    M = compact3d_system(pos).to(dtype)
    G = affine_gradient_matrix(pos).to(dtype)
    n = u_src.shape[0]
    rhs = [u_src.reshape(n, 12)]
    for (a, b) in _STRAIN_ORDER:
        rhs.append(S_src[:, :, a, b] @ G.t())     # (n, 3): x, y, z
    rhs = torch.cat(rhs, dim=1)                    # (n, 30)
    theta = torch.linalg.solve(M, rhs.t())         # (30, n)
    bt = torch.tensor(_basis3(target), dtype=dtype)
    return torch.stack([bt @ theta[m * 10:(m + 1) * 10] for m in range(3)], 1)


def _bilinear_rows(pos, dtype=torch.float64):
    return torch.tensor([[1.0, float(p[0]), float(p[1]), float(p[0]) * float(p[1])]
                         for p in pos], dtype=dtype)


def bilinear_centre_gradient_matrix(pos, dtype=torch.float64):
    """G (2, 4): gradient of the bilinear interpolant through the four square
    corners, evaluated at the centroid of the corners."""
    A = _bilinear_rows(pos, dtype)
    C = torch.linalg.inv(A)                        # coefs = C @ values
    cx = sum(float(p[0]) for p in pos) / 4.0
    cy = sum(float(p[1]) for p in pos) / 4.0
    gx = C[1] + cy * C[3]
    gy = C[2] + cx * C[3]
    return torch.stack([gx, gy], 0)


def compact2d(pos, target, u_src, S_src):
    """Quadratic compact interpolation in 2D (reading in the module header).

    pos (4, 2), target (2,), u_src (n, 4, 2), S_src (n, 4, 2, 2) -> (n, 2)."""
    dtype = u_src.dtype
    G = bilinear_centre_gradient_matrix(pos).to(dtype)
    # unknowns: u_x: [xx, yy, xy] -> 0,1,2 ; u_y: [xx, yy, xy] -> 3,4,5
    # u_x = ... + q0 x^2 + q1 y^2 + q2 xy ; u_y = ... + q3 x^2 + q4 y^2 + q5 xy
    hess = {0: [[2, 0], [0, 0]], 1: [[0, 0], [0, 2]], 2: [[0, 1], [1, 0]]}
    A = torch.zeros((6, 6), dtype=dtype)
    rhs = []
    r = 0
    for (a, b) in ((0, 0), (1, 1), (0, 1)):
        grad = S_src[:, :, a, b] @ G.t()           # (n, 2)
        for g in range(2):
            for j in range(3):
                A[r, b * 3 + j] += 0.5 * hess[j][g][a]
                A[r, a * 3 + j] += 0.5 * hess[j][g][b]
            rhs.append(grad[:, g])
            r += 1
    qc = torch.linalg.solve(A, torch.stack(rhs, 0))   # (6, n)

    def Q(p):
        x, y = float(p[0]), float(p[1])
        v = torch.tensor([x * x, y * y, x * y], dtype=dtype)
        return torch.stack([v @ qc[0:3], v @ qc[3:6]], 1)   # (n, 2)

    w = linear_weights(pos, target).to(dtype)
    out = Q(target)
    for k in range(4):
        out = out + w[k] * (u_src[:, k, :] - Q(pos[k]))
    return out


def linear_weights(pos, target, dtype=torch.float64):
    """Weights reproducing the linear (3D: 1, x, y, z) or bilinear
    (2D: 1, x, y, xy) functions at ``target`` from the four sources."""
    if len(pos[0]) == 3:
        A = torch.tensor([[1.0] + [float(v) for v in p] for p in pos], dtype=dtype)
        b = torch.tensor([1.0] + [float(v) for v in target], dtype=dtype)
    else:
        A = _bilinear_rows(pos, dtype)
        b = _bilinear_rows([target], dtype)[0]
    return torch.linalg.solve(A.t(), b)


def fill(f_src, pos, target, omega_s, omega_t, dt_ratio, lat, u_scale=1.0,
         drho_scale=1.0, rho0=1.0):
    """Steps 1-5 of Sec. 2.2 for a group of ghosts sharing one source
    geometry.

    f_src (4, q, n) pre-collision pdfs of the four sources of each ghost,
    pos (4, d) source coordinates in source-level units, target (d,),
    dt_ratio = dt_target / dt_source.  u_scale and drho_scale take the
    interpolated velocity and density deviation rho - rho0 from source to
    target lattice units (1 under acoustic scaling, where both are level
    invariant).  Returns the ghost pdfs (q, n)."""
    d = lat.d
    rhos, us, Ss, fneqs = [], [], [], []
    for k in range(4):                                   # Step 1
        rho, u, S, fneq = physics.strain_rate(f_src[k], omega_s, lat)
        rhos.append(rho)
        us.append(u.t())
        Ss.append(S.permute(2, 0, 1))
        fneqs.append(fneq)
    u_src = torch.stack(us, 1)                            # (n, 4, d)
    S_src = torch.stack(Ss, 1)                            # (n, 4, d, d)
    if d == 3:                                            # Step 2
        u_t = compact3d(pos, target, u_src, S_src)
    else:
        u_t = compact2d(pos, target, u_src, S_src)
    w = linear_weights(pos, target).to(f_src.dtype)
    rho_t = sum(w[k] * rhos[k] for k in range(4))
    fneq_t = sum(w[k] * fneqs[k] for k in range(4))
    if u_scale != 1.0 or drho_scale != 1.0:              # units of the target
        u_t = u_t * u_scale
        rho_t = rho0 + (rho_t - rho0) * drho_scale
    feq_t = physics.equilibrium(rho_t, u_t.t(), lat)      # Step 3
    fneq_t = fneq_t * (omega_s / omega_t) * dt_ratio      # Step 4
    return feq_t + fneq_t                                 # Step 5
