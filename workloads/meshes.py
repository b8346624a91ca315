"""Synthetic octree meshes given as leaf treeIDs (inputs only).

Every generator returns a :class:`MeshSpec`: the leaf treeIDs of all fluid
elements (unsorted order is allowed by the consumers; these are emitted in
slab order), the treeIDs of solid finest-level cells, the domain box in
coarsest-level cells and one boundary kind per box face.

Shapes follow the paper's workloads: the periodic Taylor-Green box with a
refined centre (Sec. 4.1), the half-refined periodic square of the TGV
convergence study (Sec. 4.1), and the sphere in a channel of size
[-15D,49D]x[-15D,15D]^2 with refinement clustered around the sphere
(Sec. 4.3).
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np

FACE_KINDS = ("periodic", "eq", "copy", "wall")


@dataclass
class MeshSpec:
    """Input description of one multilevel mesh.

    stencil     "D2Q9", "D3Q19" or "D3Q27"
    level0      coarsest level present; the root cube spans 2**level0 cells
    leaf_ids    uint64 treeIDs of all fluid leaves (any order)
    solid_ids   uint64 treeIDs of solid cells (finest level)
    box_origin  domain box origin, in level0 cells (d entries)
    box_extent  domain box extent, in level0 cells (d entries)
    face_bc     one kind per face, ordered x-, x+, y-, y+[, z-, z+]
    """
    name: str
    stencil: str
    level0: int
    leaf_ids: np.ndarray
    solid_ids: np.ndarray
    box_origin: tuple
    box_extent: tuple
    face_bc: tuple
    meta: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return 2 if self.stencil == "D2Q9" else 3


# ----------------------------------------------------------------------------
# treeID encoding (input side only)
# ----------------------------------------------------------------------------

def _level_first_id(level: int, d: int) -> int:
    return ((1 << (d * level)) - 1) // ((1 << d) - 1)


def _dilate(v: np.ndarray, d: int) -> np.ndarray:
    """Spread the bits of v (< 2^21 in 3D, < 2^32 in 2D) d positions apart."""
    v = v.astype(np.uint64)
    if d == 3:
        steps = ((32, 0x1F00000000FFFF), (16, 0x1F0000FF0000FF), (8, 0x100F00F00F00F00F),
                 (4, 0x10C30C30C30C30C3), (2, 0x1249249249249249))
        v &= np.uint64(0x1FFFFF)
    else:
        steps = ((16, 0x0000FFFF0000FFFF), (8, 0x00FF00FF00FF00FF), (4, 0x0F0F0F0F0F0F0F0F),
                 (2, 0x3333333333333333), (1, 0x5555555555555555))
        v &= np.uint64(0xFFFFFFFF)
    for sh, mask in steps:
        v = (v | (v << np.uint64(sh))) & np.uint64(mask)
    return v


def _interleave(coords: np.ndarray, level: int) -> np.ndarray:
    """Morton code of integer coords (n, d) below 2^level; x bit lowest."""
    n, d = coords.shape
    assert level <= (21 if d == 3 else 32)
    out = np.zeros(n, dtype=np.uint64)
    for a in range(d):
        out |= _dilate(coords[:, a], d) << np.uint64(a)
    return out


def encode_tree_ids(level: int, coords: np.ndarray) -> np.ndarray:
    coords = np.asarray(coords, dtype=np.int64)
    if coords.ndim == 1:
        coords = coords[None, :]
    d = coords.shape[1]
    return np.uint64(_level_first_id(level, d)) + _interleave(coords, level)


# ----------------------------------------------------------------------------
# generic nested-box generator
# ----------------------------------------------------------------------------

def _box_cells(lo: Sequence[int], hi: Sequence[int]) -> np.ndarray:
    axes = [np.arange(l, h, dtype=np.int64) for l, h in zip(lo, hi)]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=1)


def _inside(cells: np.ndarray, lo, hi) -> np.ndarray:
    m = np.ones(len(cells), dtype=bool)
    for a in range(cells.shape[1]):
        m &= (cells[:, a] >= lo[a]) & (cells[:, a] < hi[a])
    return m


def nested_mesh(name: str, stencil: str, level0: int, extent: Sequence[int],
                boxes: Sequence[tuple], face_bc: Sequence[str],
                solid: Optional[Callable[[np.ndarray], np.ndarray]] = None,
                slab: int = 16, meta: Optional[dict] = None) -> MeshSpec:
    """Leaves of a mesh refined on nested boxes.

    extent      domain size in level0 cells (origin 0)
    boxes       boxes[k] = (lo, hi) of the region refined to level0+k+1,
                given in cells of level level0+k (the level it refines)
    solid       optional predicate on finest-level integer coords; true cells
                become solid instead of fluid
    """
    d = 2 if stencil == "D2Q9" else 3
    assert len(extent) == d and len(face_bc) == 2 * d
    assert all(k in FACE_KINDS for k in face_bc)
    assert max(extent) <= (1 << level0)
    regions = [((0,) * d, tuple(extent))]
    for (lo, hi) in boxes:
        regions.append((tuple(2 * v for v in lo), tuple(2 * v for v in hi)))
    # the refinement box of level k+1 is stored in level-(k+1) cells now
    lmax = level0 + len(boxes)

    def slab_ids(k, x0, x1):
        lo, hi = regions[k]
        level = level0 + k
        cells = _box_cells((x0,) + tuple(lo[1:]), (x1,) + tuple(hi[1:]))
        if k + 1 < len(regions):
            flo, fhi = regions[k + 1]
            # a cell is refined if it lies inside the next box
            # (boxes are given on this level's grid, doubled above)
            plo = tuple(v // 2 for v in flo)
            phi = tuple(v // 2 for v in fhi)
            cells = cells[~_inside(cells, plo, phi)]
        sol = None
        if level == lmax and solid is not None:
            s = solid(cells)
            if s.any():
                sol = encode_tree_ids(level, cells[s])
            cells = cells[~s]
        return (encode_tree_ids(level, cells) if len(cells) else None), sol

    # each region is enumerated in slabs along x to bound memory; slabs are
    # independent, so a thread pool works on them (numpy releases the GIL)
    tasks = [(k, x0, min(hi[0], x0 + slab)) for k, (lo, hi) in enumerate(regions)
             for x0 in range(lo[0], hi[0], slab)]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
        parts = list(ex.map(lambda t: slab_ids(*t), tasks))
    leaf_chunks = [p[0] for p in parts if p[0] is not None]
    solid_chunks = [p[1] for p in parts if p[1] is not None]
    leaves = np.concatenate(leaf_chunks) if leaf_chunks else np.zeros(0, np.uint64)
    solids = (np.concatenate(solid_chunks) if solid_chunks
              else np.zeros(0, np.uint64))
    return MeshSpec(name=name, stencil=stencil, level0=level0, leaf_ids=leaves,
                    solid_ids=solids, box_origin=(0,) * d,
                    box_extent=tuple(extent), face_bc=tuple(face_bc),
                    meta=dict(meta or {}))


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def partition_example() -> MeshSpec:
    """The quadtree of the domain-decomposition figure (Sec. 3.1).

    The left half of the unit square is refined to level 2, the right half
    stays at level 1; the element numbers printed in the figure are the
    treeIDs listed here.
    """
    ids = np.array([13, 2, 8, 5, 16, 4, 6, 15, 7, 14], dtype=np.uint64)
    return MeshSpec(name="partition_example", stencil="D2Q9", level0=1,
                    leaf_ids=ids, solid_ids=np.zeros(0, np.uint64),
                    box_origin=(0, 0), box_extent=(2, 2),
                    face_bc=("periodic",) * 4)


def uniform_box_mesh(stencil: str, level0: int) -> MeshSpec:
    """Single-level periodic box of 2**level0 cells per axis."""
    d = 2 if stencil == "D2Q9" else 3
    n = 1 << level0
    return nested_mesh(f"uniform_{stencil}_{n}", stencil, level0, (n,) * d,
                       [], ("periodic",) * (2 * d))


def refined_box_mesh(stencil: str, level0: int, lo: int, hi: int,
                     extra_levels: Sequence[tuple] = ()) -> MeshSpec:
    """Periodic box 2**level0 per axis with the centre cube [lo,hi)^d
    refined once (and optionally nested deeper boxes, each given in the
    cells of the level it refines)."""
    d = 2 if stencil == "D2Q9" else 3
    n = 1 << level0
    boxes = [((lo,) * d, (hi,) * d)] + [((a,) * d, (b,) * d)
                                        for a, b in extra_levels]
    return nested_mesh(f"refbox_{stencil}_{n}_{lo}_{hi}", stencil, level0,
                       (n,) * d, boxes, ("periodic",) * (2 * d),
                       meta={"refine": (lo, hi)})


def half_refined_2d(level: int) -> MeshSpec:
    """Periodic square of 2**level cells whose right half is refined once
    (the Taylor-Green convergence meshes, Sec. 4.1)."""
    n = 1 << level
    return nested_mesh(f"half_refined_{n}", "D2Q9", level, (n, n),
                       [((n // 2, 0), (n, n))], ("periodic",) * 4)


def sphere_channel_mesh(d_finest: int, n_levels: int, *,
                        l0_per_d: Optional[int] = None,
                        length=(-15.0, 49.0), half_width=15.0,
                        boxes_in_d=((-5.0, 19.0, 5.0), (-2.5, 9.5, 2.5),
                                    (-1.25, 4.75, 1.25)),
                        inflow_only_eq: bool = False, outlet: str = "copy",
                        stencil: str = "D3Q19") -> MeshSpec:
    """Channel [-15D,49D]x[-15D,15D]^2 with a sphere of diameter D at the
    origin and nested refinement boxes around it (Sec. 4.3 geometry).

    d_finest    sphere diameter in finest-level cells
    n_levels    number of levels; box k (k>=1) is
                [xlo*D, xhi*D] x [-h*D, h*D]^2 from ``boxes_in_d``
    Faces: inflow x- and the four lateral faces carry the free-stream
    equilibrium; the outlet x+ copies its own post-collision values
    (outlet="copy") or also carries the free-stream equilibrium
    (outlet="eq").  The sphere centre sits on a vertex of the finest grid.
    stencil     "D3Q19" or "D3Q27"
    """
    assert 1 <= n_levels <= 1 + len(boxes_in_d)
    ratio = 1 << (n_levels - 1)
    assert d_finest % ratio == 0
    dl0 = d_finest // ratio if l0_per_d is None else l0_per_d
    ext = (int(round((length[1] - length[0]) * dl0)),
           int(round(2 * half_width * dl0)), int(round(2 * half_width * dl0)))
    level0 = int(np.ceil(np.log2(max(ext))))
    off = (-length[0], half_width, half_width)  # origin shift in D units
    boxes = []
    for k in range(1, n_levels):
        xlo, xhi, h = boxes_in_d[k - 1]
        dk = dl0 << (k - 1)  # cells per D on the level being refined
        lo = (int(round((xlo + off[0]) * dk)), int(round((-h + off[1]) * dk)),
              int(round((-h + off[2]) * dk)))
        hi = (int(round((xhi + off[0]) * dk)), int(round((h + off[1]) * dk)),
              int(round((h + off[2]) * dk)))
        boxes.append((lo, hi))
    centre = np.array([off[0] * d_finest, off[1] * d_finest, off[2] * d_finest])
    r2 = (0.5 * d_finest) ** 2

    def solid(cells: np.ndarray) -> np.ndarray:
        p = cells.astype(np.float64) + 0.5 - centre
        return (p * p).sum(axis=1) < r2

    assert outlet in ("copy", "eq")
    faces = ("eq", outlet, "eq", "eq", "eq", "eq")
    if inflow_only_eq:
        faces = ("eq", outlet, "periodic", "periodic", "periodic", "periodic")
    assert stencil in ("D3Q19", "D3Q27")
    return nested_mesh(f"sphere_D{d_finest}_L{n_levels}", stencil, level0, ext,
                       boxes, faces, solid=solid,
                       meta={"D": d_finest, "centre_finest": tuple(centre),
                             "n_levels": n_levels})


# ----------------------------------------------------------------------------
# wall fractions of links into solid cells (geometry of curved walls)
# ----------------------------------------------------------------------------
# A link from a fluid element along lattice velocity c_i into a solid cell is
# described by (treeID of the fluid element, i, q): q in [0, 1] is the
# fraction of the link, from the element's centre, at which the wall surface
# cuts it.  The velocity set ``c`` (q x d integers) is the caller's, so the
# direction indices mean what the consumer's lattice says.

def plane_channel_mesh(stencil: str, level0: int, width: int, height: int) -> MeshSpec:
    """Single-level channel: periodic along the first d-1 axes (``width``
    cells each) and ``height`` cells along the last axis, whose first and
    last cell rows are solid."""
    d = 2 if stencil == "D2Q9" else 3
    ext = (width,) * (d - 1) + (height,)

    def solid(cells):
        z = cells[:, d - 1]
        return (z == 0) | (z == height - 1)

    return nested_mesh(f"channel_{stencil}_{width}x{height}", stencil, level0, ext, [],
                       ("periodic",) * (2 * d), solid=solid,
                       meta={"height": height, "level": level0})


def two_level_channel_mesh(stencil: str, level0: int, width: int, height: int) -> MeshSpec:
    """Two-level channel: periodic along x (and z in 3D, ``width`` cells
    each), wall faces (halfway bounce-back) at y = 0 and y = ``height``; the
    upper half y >= height/2 is refined once across the whole periodic
    extent, so the lower wall touches level0 and the upper wall level0+1,
    and the level interface runs parallel to the walls."""
    d = 2 if stencil == "D2Q9" else 3
    ext = (width, height) + ((width,) if d == 3 else ())
    faces = ("periodic", "periodic", "wall", "wall") + (("periodic",) * 2 if d == 3 else ())
    lo = (0, height // 2) + ((0,) if d == 3 else ())
    hi = ext
    return nested_mesh(f"channel2_{stencil}_{width}x{height}", stencil, level0, ext,
                       [(lo, hi)], faces, meta={"height": height, "width": width})


def plane_wall_links(spec: MeshSpec, c: np.ndarray, q_low: float, q_high: float):
    """Links of a ``plane_channel_mesh`` into its solid rows; the lower wall
    cuts every link at fraction q_low, the upper at q_high (planar walls at
    z = 1.5 - q_low and z = height - 1.5 + q_high in cell units, cell
    centres at integer + 0.5)."""
    d = spec.dim
    h, L = spec.meta["height"], spec.meta["level"]
    w = spec.box_extent[0]
    lat = np.asarray(c, dtype=np.int64)
    ids, dirs, qs = [], [], []
    axes = [np.arange(w)] * (d - 1)
    grid = np.stack([g.ravel() for g in np.meshgrid(*axes, indexing="ij")], 1) \
        if d > 1 else np.zeros((1, 0), np.int64)
    for row, sgn, qv in ((1, -1, q_low), (h - 2, 1, q_high)):
        cells = np.concatenate([grid, np.full((len(grid), 1), row)], 1)
        tid = encode_tree_ids(L, cells)
        for i in range(len(lat)):
            if lat[i, d - 1] == sgn:
                ids.append(tid)
                dirs.append(np.full(len(tid), i, np.int32))
                qs.append(np.full(len(tid), qv))
    return (np.concatenate(ids), np.concatenate(dirs), np.concatenate(qs))


def sphere_wall_links(spec: MeshSpec, c: np.ndarray):
    """Links of a ``sphere_channel_mesh`` into the sphere, with the fraction
    at which the sphere surface cuts each (ray from the fluid cell's centre
    along c_i; the cell's centre lies outside, the solid neighbour's inside,
    so the first crossing is in [0, 1))."""
    d = 3
    lmax = spec.level0 + spec.meta["n_levels"] - 1
    centre = np.asarray(spec.meta["centre_finest"], dtype=np.float64)
    r = 0.5 * spec.meta["D"]
    lo = np.floor(centre - r - 2).astype(np.int64)
    hi = np.ceil(centre + r + 2).astype(np.int64)
    cells = _box_cells(tuple(lo), tuple(hi))
    a = cells.astype(np.float64) + 0.5 - centre
    fluid = (a * a).sum(1) >= r * r
    cells, a = cells[fluid], a[fluid]
    tid = encode_tree_ids(lmax, cells)
    ids = spec.leaf_ids
    ids = ids[(ids >= tid.min()) & (ids <= tid.max())]   # cheap pre-filter for big meshes
    leaf = np.isin(tid, ids)
    cells, a, tid = cells[leaf], a[leaf], tid[leaf]
    lat = np.asarray(c, dtype=np.float64)
    ids, dirs, qs = [], [], []
    for i in range(len(lat)):
        ci = lat[i]
        if not ci.any():
            continue
        b = a + ci
        hit = (b * b).sum(1) < r * r
        if not hit.any():
            continue
        aa = a[hit]
        A = float(ci @ ci)
        B = aa @ ci
        C = (aa * aa).sum(1) - r * r
        t = (-B - np.sqrt(np.maximum(B * B - A * C, 0.0))) / A
        ids.append(tid[hit])
        dirs.append(np.full(int(hit.sum()), i, np.int32))
        qs.append(np.clip(t, 0.0, 1.0))
    return (np.concatenate(ids), np.concatenate(dirs), np.concatenate(qs))
