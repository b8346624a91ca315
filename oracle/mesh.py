"""Level-wise element lists and index tables (Sec. 2.2, Sec. 3.2).

From the leaf treeIDs this builds, for every level L:

* the element list in the order [fluid | GhostFromCoarser inner |
  GhostFromCoarser outer | GhostFromFiner], each part ascending by treeID
  (Sec. 3.2 stores fluid first, then ghosts, each along the space-filling
  curve; the split of the ghost part is the reading taken here so that the
  elements a kernel updates form a prefix);
* the pull-neighbour table nbr[i][x] = index of the element at x - c_i, or
  a boundary code;
* the four interpolation sources of every ghost.

Readings taken where the paper is silent:

* GhostFromCoarser (level L > L0): every position on level L that is not
  fluid, not refined further and not solid, inside the domain, whose
  L-infinity distance to a level-L fluid element is at most m, the number
  of layers: distances 1 .. m-1 form the inner part (updated on the first
  fine step after a fill), distance m the outer layer.  m fine steps per
  coarse step consume m layers (Sec. 2.2, last paragraph): m = 2 under
  acoustic scaling (the default), m = 4 under diffusive scaling.  Its
  parent must be level-(L-1) fluid.
* GhostFromFiner (level L < Lmax): every refined level-L position within
  L-infinity distance 1 of a level-L fluid element.
* GhostFromCoarser sources (coarse level): with the ghost's octant signs s,
  H = parent, K = parent + (s_x, s_y, 0), M = parent + (s_x, 0, s_z),
  N = parent + (0, s_y, s_z); in 2D the four corners parent,
  parent + (s_x, 0), parent + (0, s_y), parent + (s_x, s_y).  Each must be
  fluid or GhostFromFiner on the coarse level.
* GhostFromFiner sources (fine level): the children at local offsets
  (0,0,0), (1,1,0), (1,0,1), (0,1,1) -- the tetrahedron H, K, M, N of
  Eq. compact_3D_u in fine units -- or all four children in 2D.  Each must be
  fluid on the fine level (GhostFromFiner takes fluid sources only).
* Boundary codes for a pull source outside the domain: the face kinds
  crossed decide, 'eq' over 'copy' over 'wall'; a solid same-level cell is
  halfway bounce-back.  A source that exists nowhere is MISSING; fluid and
  inner-layer elements may not have one.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import product
from typing import List

import numpy as np

from . import lattice as lat_mod
from . import treeid

BOUNCE = -1
EQ = -2
COPY = -3
MISSING = -4


class MeshError(ValueError):
    pass


@dataclass
class LevelTables:
    level: int
    coords: np.ndarray          # (N, d) int64, layout order
    tid: np.ndarray             # (N,) uint64
    n_fluid: int
    n_inner: int
    n_outer: int
    n_gff: int
    nbr: np.ndarray             # (q, N) int64; nbr[0] is the element itself
    gfc_src: np.ndarray         # (n_inner + n_outer, 4) indices on level L-1
    gfc_sign: np.ndarray        # (n_inner + n_outer, d) in {-1, +1}
    gff_src: np.ndarray         # (n_gff, 4) indices on level L+1
    solid_keys: np.ndarray = field(default=None)

    @property
    def n(self) -> int:
        return len(self.tid)

    @property
    def gfc_begin(self) -> int:
        return self.n_fluid

    @property
    def gff_begin(self) -> int:
        return self.n_fluid + self.n_inner + self.n_outer


@dataclass
class Mesh:
    stencil: str
    lattice: lat_mod.Lattice
    level0: int
    levels: List[LevelTables]
    box_origin: tuple
    box_extent: tuple
    face_bc: tuple

    @property
    def d(self) -> int:
        return self.lattice.d

    @property
    def lmax(self) -> int:
        return self.level0 + len(self.levels) - 1

    def lev(self, L: int) -> LevelTables:
        return self.levels[L - self.level0]

    def positions(self, L: int) -> np.ndarray:
        """Barycentres of level-L elements in level0 cell units."""
        t = self.lev(L)
        return (t.coords + 0.5) / float(1 << (L - self.level0))

    def source_sets(self, L: int) -> np.ndarray:
        """Sorted indices of level-L elements read as interpolation sources
        (by GhostFromCoarser of L+1 or GhostFromFiner of L-1)."""
        parts = []
        if L < self.lmax:
            parts.append(self.lev(L + 1).gfc_src.ravel())
        if L > self.level0:
            parts.append(self.lev(L - 1).gff_src.ravel())
        if not parts:
            return np.zeros(0, np.int64)
        return np.unique(np.concatenate(parts))


# ----------------------------------------------------------------------------

class _Geometry:
    def __init__(self, d, level0, origin, extent, faces):
        self.d, self.level0 = d, level0
        self.origin = np.array(origin, dtype=np.int64)
        self.extent = np.array(extent, dtype=np.int64)
        self.faces = faces
        self.periodic = [faces[2 * a] == "periodic" for a in range(d)]
        for a in range(d):
            if (faces[2 * a] == "periodic") != (faces[2 * a + 1] == "periodic"):
                raise MeshError("periodic faces must come in pairs")

    def lo(self, L):
        return self.origin << (L - self.level0)

    def hi(self, L):
        return (self.origin + self.extent) << (L - self.level0)

    def wrap(self, c, L):
        """Wrap periodic axes; returns (coords, outside-mask per face)."""
        c = c.copy()
        lo, hi = self.lo(L), self.hi(L)
        out_face = np.zeros((len(c), 2 * self.d), dtype=bool)
        for a in range(self.d):
            if self.periodic[a]:
                c[:, a] = lo[a] + np.mod(c[:, a] - lo[a], hi[a] - lo[a])
            else:
                out_face[:, 2 * a] = c[:, a] < lo[a]
                out_face[:, 2 * a + 1] = c[:, a] >= hi[a]
        return c, out_face

    def key(self, c, L):
        k = np.zeros(len(c), dtype=np.int64)
        for a in reversed(range(self.d)):
            k = k * (np.int64(1) << L) + c[:, a]
        return k


def _isin(keys, sorted_set):
    if len(sorted_set) == 0:
        return np.zeros(len(keys), dtype=bool)
    pos = np.searchsorted(sorted_set, keys)
    pos = np.minimum(pos, len(sorted_set) - 1)
    return sorted_set[pos] == keys


def build(spec, gfc_layers: int = 2) -> Mesh:
    """Build all tables from a workloads.MeshSpec; gfc_layers GhostFromCoarser
    layers (2: acoustic scaling, 4: diffusive scaling)."""
    if gfc_layers < 2:
        raise MeshError("at least two GhostFromCoarser layers")
    lat = lat_mod.get(spec.stencil)
    d = lat.d
    geo = _Geometry(d, spec.level0, spec.box_origin, spec.box_extent,
                    tuple(spec.face_bc))
    lv, lc = treeid.decode(spec.leaf_ids, d)
    sv, sc = treeid.decode(spec.solid_ids, d)
    if len(lv) == 0:
        raise MeshError("no leaves")
    L0 = spec.level0
    if lv.min() < L0 or (len(sv) and sv.min() < L0):
        raise MeshError("element coarser than level0")
    lmax = int(max(lv.max(), sv.max() if len(sv) else 0))
    # every element inside the domain box
    for levs, cs in ((lv, lc), (sv, sc)):
        for L in np.unique(levs):
            m = levs == L
            lo, hi = geo.lo(int(L)), geo.hi(int(L))
            if ((cs[m] < lo) | (cs[m] >= hi)).any():
                raise MeshError("element outside the domain box")
    # coverage: leaves and solids tile the box exactly (overlaps checked below)
    vol = float(np.sum(2.0 ** (-d * (lv - L0).astype(np.float64)))) + \
        float(np.sum(2.0 ** (-d * (sv - L0).astype(np.float64))))
    if abs(vol - float(np.prod(geo.extent))) > 1e-9:
        raise MeshError("leaves do not tile the domain box")

    fluid, solid, refined = {}, {}, {}
    for L in range(L0, lmax + 1):
        fk = np.sort(geo.key(lc[lv == L], L))
        if len(fk) and (np.diff(fk) == 0).any():
            raise MeshError("duplicate leaf")
        fluid[L] = fk
        solid[L] = np.sort(geo.key(sc[sv == L], L))
        anc = []
        for levs, cs in ((lv, lc), (sv, sc)):
            m = levs > L
            if m.any():
                anc.append(geo.key(cs[m] >> (levs[m] - L)[:, None], L))
        refined[L] = np.unique(np.concatenate(anc)) if anc else np.zeros(0, np.int64)
        if _isin(fk, refined[L]).any() or _isin(solid[L], refined[L]).any() \
                or _isin(fk, solid[L]).any():
            raise MeshError("overlapping elements")

    def coords_of(keys, L):
        out = np.zeros((len(keys), d), dtype=np.int64)
        k = keys.copy()
        for a in range(d):
            out[:, a] = k & ((np.int64(1) << L) - 1)
            k = k >> L
        return out

    # ---- ghost classification --------------------------------------------
    gff_keys, gfc_inner, gfc_outer = {}, {}, {}
    for L in range(L0, lmax + 1):
        fc = coords_of(fluid[L], L)
        # GhostFromFiner
        cand = []
        if L < lmax:
            for off in product((-1, 0, 1), repeat=d):
                if not any(off):
                    continue
                c, out = geo.wrap(fc + np.array(off), L)
                ok = ~out.any(1)
                k = geo.key(c[ok], L)
                cand.append(k[_isin(k, refined[L])])
        gff_keys[L] = np.unique(np.concatenate(cand)) if cand else np.zeros(0, np.int64)
        # GhostFromCoarser
        inner, outer = [], []
        if L > L0:
            occupied = np.unique(np.concatenate([fluid[L], refined[L], solid[L]]))
            m = gfc_layers
            for off in product(range(-m, m + 1), repeat=d):
                if not any(off):
                    continue
                dist = max(abs(o) for o in off)
                c, out = geo.wrap(fc + np.array(off), L)
                ok = ~out.any(1)
                k = geo.key(c[ok], L)
                k = k[~_isin(k, occupied)]
                (inner if dist < m else outer).append(k)
        ik = np.unique(np.concatenate(inner)) if inner else np.zeros(0, np.int64)
        ok_ = np.unique(np.concatenate(outer)) if outer else np.zeros(0, np.int64)
        ok_ = ok_[~_isin(ok_, ik)]
        gfc_inner[L], gfc_outer[L] = ik, ok_

    # ---- layout -------------------------------------------------------------
    layout = {}
    for L in range(L0, lmax + 1):
        parts = []
        for keys in (fluid[L], gfc_inner[L], gfc_outer[L], gff_keys[L]):
            c = coords_of(keys, L)
            t = treeid.encode(L, c) if len(c) else np.zeros(0, np.uint64)
            o = np.argsort(t, kind="stable")
            parts.append((c[o], t[o]))
        layout[L] = parts

    levels = []
    for L in range(L0, lmax + 1):
        parts = layout[L]
        coords = np.concatenate([p[0] for p in parts])
        tid = np.concatenate([p[1] for p in parts])
        n_f, n_i, n_o, n_g = (len(p[0]) for p in parts)
        keys = geo.key(coords, L)
        korder = np.argsort(keys)
        ksorted = keys[korder]

        def lookup(kq, ksorted=ksorted, korder=korder):
            pos = np.searchsorted(ksorted, kq)
            pos = np.minimum(pos, max(len(ksorted) - 1, 0))
            hit = ksorted[pos] == kq if len(ksorted) else np.zeros(len(kq), bool)
            return np.where(hit, korder[pos], -1)

        N = len(tid)
        nbr = np.zeros((lat.q, N), dtype=np.int64)
        for i in range(lat.q):
            c, out = geo.wrap(coords - lat.c[i], L)
            idx = np.full(N, MISSING, dtype=np.int64)
            inside = ~out.any(1)
            kin = geo.key(c[inside], L)
            found = lookup(kin)
            sub = np.full(inside.sum(), MISSING, dtype=np.int64)
            sub[found >= 0] = found[found >= 0]
            sub[(found < 0) & _isin(kin, solid[L])] = BOUNCE
            idx[inside] = sub
            # faces crossed
            if (~inside).any():
                face_kinds = np.array(geo.faces)
                o = out[~inside]
                code = np.full(len(o), BOUNCE, dtype=np.int64)
                has_copy = (o & (face_kinds == "copy")[None, :]).any(1)
                has_eq = (o & (face_kinds == "eq")[None, :]).any(1)
                code[has_copy] = COPY
                code[has_eq] = EQ
                idx[~inside] = code
            nbr[i] = idx
        # active elements may not miss a neighbour
        act = n_f + n_i
        if (nbr[:, :act] == MISSING).any():
            bad = np.where((nbr[:, :act] == MISSING).any(0))[0][0]
            raise MeshError(f"level {L}: active element {tid[bad]} lacks a neighbour")
        levels.append(dict(L=L, coords=coords, tid=tid, n=(n_f, n_i, n_o, n_g),
                           nbr=nbr, lookup=lookup))

    # ---- interpolation sources ----------------------------------------------
    if d == 3:
        gff_child = np.array([(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)])
    else:
        gff_child = np.array([(0, 0), (1, 0), (0, 1), (1, 1)])
    out_levels = []
    for li, L in enumerate(range(L0, lmax + 1)):
        e = levels[li]
        n_f, n_i, n_o, n_g = e["n"]
        coords = e["coords"]
        # GhostFromFiner sources on level L+1
        gff_src = np.zeros((n_g, 4), dtype=np.int64)
        if n_g:
            fine = levels[li + 1]
            gc = coords[n_f + n_i + n_o:]
            for k in range(4):
                ch = 2 * gc + gff_child[k]
                idx = fine["lookup"](geo.key(ch, L + 1))
                if (idx < 0).any() or (idx >= fine["n"][0]).any():
                    raise MeshError(f"level {L}: GhostFromFiner source is not fluid")
                gff_src[:, k] = idx
        # GhostFromCoarser sources on level L-1
        ng = n_i + n_o
        gfc_src = np.zeros((ng, 4), dtype=np.int64)
        gfc_sign = np.zeros((ng, d), dtype=np.int64)
        if ng:
            coarse = levels[li - 1]
            cf, ci, co, cg = coarse["n"]
            gc = coords[n_f:n_f + ng]
            parent = gc >> 1
            s = 2 * (gc & 1) - 1
            gfc_sign[:] = s
            if d == 3:
                offs = [np.zeros_like(s), s * np.array([1, 1, 0]),
                        s * np.array([1, 0, 1]), s * np.array([0, 1, 1])]
            else:
                offs = [np.zeros_like(s), s * np.array([1, 0]),
                        s * np.array([0, 1]), s * np.array([1, 1])]
            for k in range(4):
                c, out = geo.wrap(parent + offs[k], L - 1)
                if out.any():
                    raise MeshError(f"level {L}: GhostFromCoarser source outside domain")
                idx = coarse["lookup"](geo.key(c, L - 1))
                okk = (idx >= 0) & ((idx < cf) | (idx >= cf + ci + co))
                if k == 0:
                    okk &= (idx >= 0) & (idx < cf)
                if not okk.all():
                    raise MeshError(f"level {L}: GhostFromCoarser source is not "
                                    "fluid or GhostFromFiner")
                gfc_src[:, k] = idx
        out_levels.append(LevelTables(
            level=L, coords=coords, tid=e["tid"], n_fluid=n_f, n_inner=n_i,
            n_outer=n_o, n_gff=n_g, nbr=e["nbr"], gfc_src=gfc_src,
            gfc_sign=gfc_sign, gff_src=gff_src, solid_keys=solid[L]))
    return Mesh(spec.stencil, lat, L0, out_levels, tuple(spec.box_origin),
                tuple(spec.box_extent), tuple(spec.face_bc))
