"""Multilevel time stepping, plain and slow (Sec. 2.1-2.3).

State: the pre-collision pdfs f of every element of every level.  One step
of level L applies the BGK collision (Eq. bgk) to *every* element of the
level and then streams: f_i(x, t+1) = f*_i(x - c_i, t).  Nothing is skipped:
ghost elements are collided too (Sec. 3.2 feeds all element types into the
compute kernel), and a pull source that does not exist yields NaN, so any
use of a value that is not valid poisons the result.

Schedule (Sec. 2.2, acoustic scaling with two fine steps per coarse step,
GhostFromFiner before GhostFromCoarser, two GhostFromCoarser layers and no
temporal interpolation); reading taken for the order:

    advance(L): step(L); if L < Lmax: advance(L+1); advance(L+1);
                fill GhostFromFiner(L); fill GhostFromCoarser(L+1)

Diffusive scaling (the variant Sec. 2.2 closes with; ``scaling="diffusive"``,
mesh built with four GhostFromCoarser layers): dt halves twice per level,
so advance(L+1) runs four times per step of L; tau is the same on every
level (nu dt/dx^2 is level invariant); the fills take the interpolated
velocity from source to target lattice units by (dt_t/dt_s)/(dx_t/dx_s)
and the density deviation by its square, and Step 4 rescales f^neq by
omega_s/omega_t times dt_t/dt_s as under acoustic scaling.  Mass and
kinetic energy are reported in level-L0 units.

Initialisation (reading taken; the paper is silent about ghosts at t=0):
fluid pdfs are f^eq(rho, u) + f^neq(S) from the given fields, then one
synchronous fill of all GhostFromFiner and then all GhostFromCoarser.

Boundary rules for pull sources: halfway bounce-back from a solid cell or
wall face takes f*_{opp(i)}(x); an 'eq' face supplies f^eq(rho0, u_in); a
'copy' face takes the element's own f*_i(x).

Curved walls (Sec. 2.3, the linear interpolated bounce-back of Bouzidi,
Firdaouss and Lallemand, 2001): a link from fluid element x along c_i into a
solid cell may carry the fraction q in [0, 1] of the link at which the wall
cuts it.  With ibar = opp(i) and x2 the element at x - c_i:

    q <  1/2: f_ibar(x, t+1) = 2q f*_i(x) + (1 - 2q) f*_i(x2)
    q >= 1/2: f_ibar(x, t+1) = f*_i(x) / (2q) + (1 - 1/(2q)) f*_ibar(x)

Both give halfway bounce-back at q = 1/2.  Reading taken: where x - c_i is
not an element (a solid cell, a face), a link with q < 1/2 falls back to
halfway bounce-back.  Links without a fraction stay halfway.
"""
from __future__ import annotations

import numpy as np
import torch

from . import interp, physics
from .mesh import BOUNCE, COPY, EQ, MISSING


class OracleSim:
    def __init__(self, mesh, tau0, rho0: float = 1.0, u_in=None,
                 poison: bool = True, dtype=torch.float64, walls=None,
                 scaling: str = "acoustic"):
        self.mesh = mesh
        self.lat = mesh.lattice
        self.dtype = dtype
        self.L0, self.Lmax = mesh.level0, mesh.lmax
        self.tau0 = tau0
        if scaling not in ("acoustic", "diffusive"):
            raise ValueError(scaling)
        # fine steps per coarse step: dt_(L+1) = dt_L / n_sub, dx_(L+1) = dx_L / 2
        self.scaling = scaling
        self.n_sub = 2 if scaling == "acoustic" else 4
        if scaling == "acoustic":
            self.omega = {L: 1.0 / physics.level_tau(tau0, L, self.L0)
                          for L in range(self.L0, self.Lmax + 1)}
        else:   # nu dt / dx^2 is the same on every level
            self.omega = {L: 1.0 / tau0 for L in range(self.L0, self.Lmax + 1)}
        self.rho0 = rho0
        d = self.lat.d
        if u_in is None:
            u_in = torch.zeros(d, dtype=dtype)
        self.u_in = torch.as_tensor(u_in, dtype=dtype)
        self.poison = poison
        self.f = {}
        self._stream_tables = {L: self._tables(L) for L in range(self.L0, self.Lmax + 1)}
        self.walls = {} if walls is None else wall_links(mesh, *walls)
        self.time = 0  # coarse steps

    # ------------------------------------------------------------------
    def _tables(self, L):
        t = self.mesh.lev(L)
        q, N = self.lat.q, t.n
        nbr = t.nbr
        x = np.arange(N)[None, :].repeat(q, 0)
        dirs = np.arange(q)[:, None].repeat(N, 1)
        src_dir = dirs.copy()
        src_elem = np.where(nbr >= 0, nbr, 0)
        bb = nbr == BOUNCE
        src_dir[bb] = self.lat.opp[dirs[bb]]
        src_elem[bb] = x[bb]
        cp = nbr == COPY
        src_elem[cp] = x[cp]
        flat = torch.from_numpy(src_dir * N + src_elem)
        return dict(flat=flat, eq=torch.from_numpy(nbr == EQ),
                    miss=torch.from_numpy(nbr == MISSING))

    def _filler(self, n):
        if self.poison:
            return torch.full((self.lat.q, n), float("nan"), dtype=self.dtype)
        return self.lat.w_t(self.dtype)[:, None].expand(self.lat.q, n).clone()

    # ------------------------------------------------------------------
    def init(self, rho, u, S):
        """rho[L] (n_fluid,), u[L] (n_fluid, d), S[L] (n_fluid, d, d) in
        level-L lattice units, for every level L."""
        for L in range(self.L0, self.Lmax + 1):
            t = self.mesh.lev(L)
            r = torch.as_tensor(rho[L], dtype=self.dtype)
            uu = torch.as_tensor(u[L], dtype=self.dtype).t()
            SS = torch.as_tensor(S[L], dtype=self.dtype).permute(1, 2, 0)
            f_fluid = physics.equilibrium(r, uu, self.lat) + \
                physics.fneq_from_strain(r, SS, self.omega[L], self.lat)
            self.f[L] = torch.cat([f_fluid, self._filler(t.n - t.n_fluid)], 1)
        self.fill_all()

    def fill_all(self):
        for L in range(self.L0, self.Lmax):
            self.fill_gff(L)
        for L in range(self.L0 + 1, self.Lmax + 1):
            self.fill_gfc(L)

    def fill_gff(self, L):
        """GhostFromFiner of level L from fluid sources on level L+1."""
        t = self.mesh.lev(L)
        if t.n_gff == 0:
            return
        d = self.lat.d
        if d == 3:
            pos = [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
        else:
            pos = [(0, 0), (1, 0), (0, 1), (1, 1)]
        target = (0.5,) * d
        fs = self.f[L + 1]
        src = torch.from_numpy(t.gff_src)
        f_src = torch.stack([fs[:, src[:, k]] for k in range(4)], 0)
        r = self.n_sub / 2.0          # (dt_c / dt_f) / (dx_c / dx_f)
        vals = interp.fill(f_src, pos, target, self.omega[L + 1], self.omega[L],
                           float(self.n_sub), self.lat, u_scale=r, drho_scale=r * r,
                           rho0=self.rho0)
        idx = torch.arange(t.gff_begin, t.n)
        self.f[L] = self.f[L].index_copy(1, idx, vals)

    def fill_gfc(self, L):
        """GhostFromCoarser (both layers) of level L from level L-1."""
        t = self.mesh.lev(L)
        ng = t.n_inner + t.n_outer
        if ng == 0:
            return
        d = self.lat.d
        fc = self.f[L - 1]
        signs = t.gfc_sign
        codes = ((signs + 1) // 2) @ (1 << np.arange(d))
        out = self.f[L]
        for oc in np.unique(codes):
            m = np.where(codes == oc)[0]
            s = signs[m[0]]
            if d == 3:
                pos = [(0, 0, 0), (s[0], s[1], 0), (s[0], 0, s[2]), (0, s[1], s[2])]
            else:
                pos = [(0, 0), (s[0], 0), (0, s[1]), (s[0], s[1])]
            target = tuple(0.25 * v for v in s)
            src = torch.from_numpy(t.gfc_src[m])
            f_src = torch.stack([fc[:, src[:, k]] for k in range(4)], 0)
            r = 2.0 / self.n_sub      # (dt_f / dt_c) / (dx_f / dx_c)
            vals = interp.fill(f_src, pos, target, self.omega[L - 1],
                               self.omega[L], 1.0 / self.n_sub, self.lat, u_scale=r,
                               drho_scale=r * r, rho0=self.rho0)
            out = out.index_copy(1, torch.from_numpy(t.gfc_begin + m), vals)
        self.f[L] = out

    # ------------------------------------------------------------------
    def feq_inflow(self):
        rho = torch.full((1,), self.rho0, dtype=self.dtype)
        return physics.equilibrium(rho, self.u_in[:, None], self.lat)[:, 0]

    def stream(self, L, fstar):
        tb = self._stream_tables[L]
        f = fstar.reshape(-1)[tb["flat"]]
        f = torch.where(tb["eq"], self.feq_inflow()[:, None].expand_as(f), f)
        f = torch.where(tb["miss"], self._filler(f.shape[1]), f)
        if L in self.walls:
            f = self.curved_walls(L, fstar, f)
        return f

    def curved_walls(self, L, fstar, f):
        """Replace the halfway bounce-back values of links that carry a wall
        fraction by the linear interpolated bounce-back (module docstring)."""
        x, i, q, x2 = self.walls[L]
        ibar = torch.from_numpy(self.lat.opp[i])
        x, i = torch.from_numpy(x), torch.from_numpy(i)
        q = torch.as_tensor(q, dtype=self.dtype)
        has2 = torch.from_numpy(x2 >= 0)
        x2 = torch.from_numpy(np.where(x2 >= 0, x2, 0))
        own = fstar[i, x]                       # f*_i(x), moving into the wall
        near = 2 * q * own + (1 - 2 * q) * fstar[i, x2]
        near = torch.where(has2, near, own)
        qf = torch.where(q >= 0.5, q, torch.ones_like(q))
        far = own / (2 * qf) + (1 - 1 / (2 * qf)) * fstar[ibar, x]
        out = f.clone()
        out[ibar, x] = torch.where(q < 0.5, near, far)
        return out

    def stream_collide(self, L):
        fstar = physics.collide(self.f[L], self.omega[L], self.lat)
        self.f[L] = self.stream(L, fstar)

    def advance(self, L):
        self.stream_collide(L)
        if L < self.Lmax:
            for _ in range(self.n_sub):
                self.advance(L + 1)
            self.fill_gff(L)
            self.fill_gfc(L + 1)

    def step(self, n: int = 1):
        for _ in range(n):
            self.advance(self.L0)
            self.time += 1

    # ------------------------------------------------------------------
    def post_collision(self, L):
        return physics.collide(self.f[L], self.omega[L], self.lat)

    def fluid_moments(self, L):
        t = self.mesh.lev(L)
        rho, u, S, _ = physics.strain_rate(self.f[L][:, :t.n_fluid],
                                           self.omega[L], self.lat)
        return rho, u, S

    def volume(self, L):
        return 2.0 ** (-self.lat.d * (L - self.L0))

    def unit_ratio(self, L):
        """Level-L0 lattice velocity per level-L lattice velocity:
        (dx_L / dt_L) / (dx_L0 / dt_L0) = (n_sub / 2)^(L - L0)."""
        return (self.n_sub / 2.0) ** (L - self.L0)

    def mass(self):
        """sum_L V_L sum_fluid rho, density deviations in level-L0 units."""
        tot = 0.0
        for L in range(self.L0, self.Lmax + 1):
            rho, _, _ = self.fluid_moments(L)
            r = self.unit_ratio(L)
            tot = tot + self.volume(L) * (self.rho0 + (rho - self.rho0) * r * r).sum()
        return tot

    def kinetic_energy(self):
        """E = 1/2 sum_L V_L sum_fluid rho |u|^2 (V_L in level0 cells, u in
        level-L0 lattice units)."""
        tot = 0.0
        for L in range(self.L0, self.Lmax + 1):
            rho, u, _ = self.fluid_moments(L)
            r = self.unit_ratio(L)
            tot = tot + self.volume(L) * 0.5 * (rho * (u * u).sum(0)).sum() * r * r
        return tot

    def force(self):
        """Momentum exchange (Sec. 2.3): F = sum_{x_b} sum_{i in V}
        c_i [f*_i(x_b, t) + f_opp(i)(x_b, t + dt)] over fluid elements x_b
        next to the solid and the directions i pointing into it.  Each level's
        sum is in its own lattice units; they are added in finest-level units
        (force scales with dx^(d-1) under acoustic scaling)."""
        if self.scaling != "acoustic":
            raise NotImplementedError("force under diffusive scaling")
        d = self.lat.d
        c = self.lat.c_t(self.dtype)
        total = torch.zeros(d, dtype=self.dtype)
        for L in range(self.L0, self.Lmax + 1):
            t = self.mesh.lev(L)
            fstar = self.post_collision(L)
            fnew = self.stream(L, fstar)
            nb = t.nbr[:, :t.n_fluid]
            ibar, x = np.where(nb == BOUNCE)   # pull source x - c_ibar is solid
            if len(x) == 0:
                continue
            i = self.lat.opp[ibar]             # c_i points into the solid
            vals = fstar[i, x] + fnew[ibar, x]
            FL = (c[i] * vals[:, None]).sum(0)
            total = total + FL * float(2 ** ((d - 1) * (self.Lmax - L)))
        return total


def wall_links(mesh, ids, dirs, q):
    """Per level, the links (x, i, q, x2) of fluid elements x (layout index)
    whose neighbour x + c_i is solid, from treeIDs, directions i pointing
    into the solid and wall fractions q in [0, 1]; x2 is the element at
    x - c_i, or a negative code where there is none."""
    ids = np.asarray(ids, dtype=np.uint64)
    dirs = np.asarray(dirs, dtype=np.int64)
    q = np.asarray(q, dtype=np.float64)
    if not (len(ids) == len(dirs) == len(q)):
        raise ValueError("wall links: sizes differ")
    if len(q) and (not np.isfinite(q).all() or q.min() < 0 or q.max() > 1):
        raise ValueError("wall fraction outside [0, 1]")
    lat = mesh.lattice
    out = {}
    for L in range(mesh.level0, mesh.lmax + 1):
        t = mesh.lev(L)
        fl = t.tid[:t.n_fluid]
        if len(fl) == 0:
            continue
        order = np.argsort(fl)
        srt = fl[order]
        pos = np.minimum(np.searchsorted(srt, ids), len(fl) - 1)
        on = srt[pos] == ids
        if not on.any():
            continue
        x = order[pos[on]]
        i = dirs[on]
        if (i < 0).any() or (i >= lat.q).any() or not np.abs(lat.c[i]).sum(1).all():
            raise ValueError("wall link direction out of range or at rest")
        ibar = lat.opp[i]
        if (t.nbr[ibar, x] != BOUNCE).any():
            raise ValueError("wall link whose neighbour is not solid")
        key = x * lat.q + i
        if len(np.unique(key)) != len(key):
            raise ValueError("wall link given twice")
        out[L] = (x, i, q[on], t.nbr[i, x])
    found = sum(len(v[0]) for v in out.values())
    if found != len(ids):
        raise ValueError("wall link on an element that is not a fluid leaf")
    return out
