"""The library's host plan (C++) against the oracle's mesh tables, bit for
bit, compared by treeID; plus C-ABI symbol exports and error paths.  CPU
only: these calls never touch a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import mesh as omesh

M = pytest.importorskip("paper_1601_06984_amd")
from paper_1601_06984_amd import _lib  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MESHES = {
    "d2q9_refbox_32": lambda: W.refined_box_mesh("D2Q9", 5, 8, 24),
    "d3q19_refbox_32": lambda: W.refined_box_mesh("D3Q19", 5, 8, 24),
    "d3q19_refbox_16": lambda: W.refined_box_mesh("D3Q19", 4, 4, 12),
    "d2q9_half_16": lambda: W.half_refined_2d(4),
    "d2q9_three_level": lambda: W.refined_box_mesh("D2Q9", 5, 8, 24, extra_levels=[(20, 44)]),
    "d3q19_three_level": lambda: W.refined_box_mesh("D3Q19", 4, 2, 14, extra_levels=[(10, 18)]),
    "d3q19_sphere_small": lambda: W.sphere_channel_mesh(8, 2, l0_per_d=4, length=(-2.0, 3.0),
                                                        half_width=2.0,
                                                        boxes_in_d=((-1.0, 1.5, 1.0),)),
    "d3q19_sphere_3lev": lambda: W.sphere_channel_mesh(8, 3, length=(-3.0, 5.0), half_width=3.0,
                                                       boxes_in_d=((-2.0, 3.0, 2.0),
                                                                   (-1.0, 2.0, 1.0))),
    "d3q27_three_level": lambda: W.refined_box_mesh("D3Q27", 4, 2, 14, extra_levels=[(10, 18)]),
    "d3q27_sphere_small": lambda: W.sphere_channel_mesh(8, 2, l0_per_d=4, length=(-2.0, 3.0),
                                                        half_width=2.0,
                                                        boxes_in_d=((-1.0, 1.5, 1.0),),
                                                        stencil="D3Q27"),
}

CODE_MAP = {omesh.BOUNCE: _lib.NBR_BOUNCE, omesh.EQ: _lib.NBR_EQ,
            omesh.COPY: _lib.NBR_COPY, omesh.MISSING: _lib.NBR_MISSING}


def _dir_perm(stencil, olat):
    c, _ = M.lattice(stencil)
    perm = []
    for i in range(len(c)):
        j = int(np.where((olat.c == c[i]).all(1))[0][0])
        perm.append(j)
    return perm


def _g2o(gt, ot):
    order = np.argsort(ot)
    pos = np.searchsorted(ot[order], gt)
    g2o = order[np.minimum(pos, len(ot) - 1)]
    assert np.array_equal(ot[g2o], gt)
    return g2o


@pytest.mark.parametrize("name", sorted(MESHES))
def test_plan_tables_bit_exact(name):
    """Every table equals the oracle's after mapping element indices through
    treeIDs.  Layout rule: [fluid | GFC inner | GFC outer | GFF] with the
    fluid part split into [not an interpolation source | source], each part
    ascending by treeID; the ghost parts coincide with the oracle's."""
    _check_tables(MESHES[name](), 2)


@pytest.mark.parametrize("spec_fn", [lambda: W.refined_box_mesh("D2Q9", 5, 8, 24),
                                     lambda: W.refined_box_mesh("D3Q19", 4, 4, 12),
                                     lambda: W.refined_box_mesh("D2Q9", 6, 12, 44,
                                                                extra_levels=[(32, 56)])])
def test_plan_tables_bit_exact_four_layers(spec_fn):
    """Diffusive-scaling plans (four GhostFromCoarser layers; distances 1-3
    inner, 4 outer) against the oracle's four-layer mesh; layer counts
    other than 2 and 4 are refused."""
    M.set_gfc_layers(4)
    try:
        plan = _check_tables(spec_fn(), 4)
    finally:
        M.set_gfc_layers(2)
    assert plan.gfc_layers == 4
    with pytest.raises(M.MLBMError):
        M.set_gfc_layers(3)


def _check_tables(spec, layers):
    om = omesh.build(spec, gfc_layers=layers)
    plan = M.Plan.from_spec(spec)
    assert plan.n_levels == len(om.levels) and plan.level0 == om.level0
    perm = _dir_perm(spec.stencil, om.lattice)
    g2o = [_g2o(plan.export(k, "treeid"), ot.tid) for k, ot in enumerate(om.levels)]
    for k, ot in enumerate(om.levels):
        info = plan.info[k]
        assert (info["n"], info["n_fluid"], info["n_gfc_inner"], info["n_gfc_outer"],
                info["n_gff"]) == (ot.n, ot.n_fluid, ot.n_inner, ot.n_outer, ot.n_gff)
        tid = plan.export(k, "treeid")
        nf, cb = ot.n_fluid, ot.n_fluid - info["n_cap_fluid"]
        # segment order and contents
        for a, b in ((0, cb), (cb, nf)):
            assert np.all(np.diff(tid[a:b].astype(np.int64)) > 0)
        assert np.array_equal(tid[nf:], ot.tid[nf:])
        src = om.source_sets(ot.level)
        src = src[src < nf]
        assert np.array_equal(np.sort(tid[cb:nf]), np.sort(ot.tid[src]))
        assert np.array_equal(plan.export(k, "capture"), np.arange(cb, nf))
        m = g2o[k]
        assert np.array_equal(plan.export(k, "coords"), ot.coords[m].T)
        nbr = plan.export(k, "nbr")
        for i in range(1, plan.q):
            o = ot.nbr[perm[i]][m]
            got = nbr[i - 1]
            mapped = np.where(got >= 0, m[np.maximum(got, 0)], got)
            want = o.copy()
            for oc, gc in CODE_MAP.items():
                want = np.where(o == oc, gc, want)
            assert np.array_equal(mapped, want), (k, i)
        ng = ot.n_inner + ot.n_outer
        if ng:
            gs = plan.export(k, "gfc_src").reshape(4, ng)
            assert np.array_equal(g2o[k - 1][gs], ot.gfc_src.T)
        if ot.n_gff:
            gs = plan.export(k, "gff_src").reshape(4, ot.n_gff)
            assert np.array_equal(g2o[k + 1][gs], ot.gff_src.T)
        b = plan.export(k, "bounce").reshape(2, -1)
        got = set(zip(m[b[0]].tolist(), b[1].tolist()))
        ob = set()
        for i in range(1, plan.q):
            xs = np.where(ot.nbr[perm[i], :ot.n_fluid] == omesh.BOUNCE)[0]
            ob.update((int(x), i) for x in xs)
        assert got == ob
    return plan


COMPRESS_MESHES = dict(MESHES)
# large enough to hold blocks whose neighbours need more than four bases
COMPRESS_MESHES["tgv64_refined"] = lambda: W.refined_box_mesh("D3Q19", 6, 16, 48)
# levels that take Morton directions under the default policy
COMPRESS_MESHES["sphere_d12"] = lambda: W.sphere_channel_mesh(12, 3, outlet="eq")
COMPRESS_MESHES["d3q19_morton"] = lambda: W.refined_box_mesh("D3Q19", 5, 14, 18)
COMPRESS_MESHES["d2q9_morton"] = lambda: W.refined_box_mesh("D2Q9", 7, 56, 72)
COMPRESS_MESHES["d3q27_morton"] = lambda: W.refined_box_mesh("D3Q27", 5, 14, 18)


def _morton_pull(m, c, d):
    """Low 32 bits of the Morton code of (cell of code m) - c: each axis
    step moves the axis's interleaved bits by one, carrying through the
    other axes' bits (the 32-bit masks of bit positions d*b + a)."""
    masks = [0x49249249, 0x92492492, 0x24924924] if d == 3 else [0x55555555, 0xAAAAAAAA]
    m = m.astype(np.uint64)
    full = np.uint64(0xFFFFFFFF)
    for a in range(d):
        s = -c[a]
        if s == 0:
            continue
        mask = np.uint64(masks[a]); one = np.uint64(1 << a)
        t = ((m | (~mask & full)) + one) if s > 0 else ((m & mask) + full + np.uint64(1) - one)
        m = ((t & mask) | (m & (~mask & full))) & full
    return m


@pytest.mark.parametrize("name", sorted(COMPRESS_MESHES))
def test_compressed_pull_table_decodes_to_the_table(name, morton):
    """The device form of the pull table (Morton directions, 16-bit codes
    against per-block bases, int32 rows for wide blocks) decodes to exactly
    the int32 table over every updated element."""
    plan = M.Plan.from_spec(COMPRESS_MESHES[name]())
    d = plan.d
    cvel, _ = M.lattice(plan.stencil)
    n_wide = n_mor = n_dir = 0
    for k, inf in enumerate(plan.info):
        nbr = plan.export(k, "nbr")
        q1 = nbr.shape[0]
        act = inf["n_fluid"] + inf["n_gfc_inner"]
        nblk = (act + 255) // 256
        c16 = plan.export(k, "nbr16").astype(np.int64)
        base = plan.export(k, "nbase").reshape(nblk, q1, 4).astype(np.int64)
        hdr = plan.export(k, "nbr_hdr").reshape(nblk, 4).astype(np.int64)
        hi = plan.export(k, "nbr_wide").astype(np.int64)
        tid = plan.export(k, "treeid")
        coords = plan.export(k, "coords")
        n_wide += int((hdr[:, 2] >= 0).sum())
        assert c16.shape == (q1, nblk * 256)
        x = np.arange(act)
        b = x // 256
        w = hdr[b, 2]
        regm = hdr[b, 0] & 0xFFFFFFFF
        m = (x + (hdr[b, 1] & 0xFFFFFFFF)) & 0xFFFFFFFF
        # the block's Morton codes are its treeIDs minus the level's first ID
        mor_blk = hdr[b, 0] != 0
        first = tid[0] - _morton_of(coords[:, :1], d, plan.level0 + k)[0]
        assert np.array_equal(m[mor_blk].astype(np.uint64),
                              (tid[:act][mor_blk] - first) & np.uint64(0xFFFFFFFF))
        for i in range(q1):
            c = c16[i, :act]
            dec = np.where(c >= 0xFFFC, c - 0x10000,
                           base[b, i, np.minimum(c >> 14, 3)] + (c & 0x3FFF))
            mor = ((regm >> (i + 1)) & 1).astype(bool)
            if mor.any():
                ci = [int(v) for v in cvel[i + 1]]
                mo = _morton_pull(m[mor], ci, d).astype(np.int64)
                bb = base[b[mor], i] & 0xFFFFFFFF
                sel = ((mo - bb[:, 2]) & 0xFFFFFFFF) >= bb[:, 3]
                src = (mo + np.where(sel, bb[:, 1], bb[:, 0])) & 0xFFFFFFFF
                dec[mor] = np.where(src >= 1 << 31, src - (1 << 32), src)
                assert (w[mor] < 0).all()
            if (w >= 0).any():
                full = (hi[i, w[w >= 0] * 256 + x[w >= 0] % 256] << 16) | c[w >= 0]
                dec[w >= 0] = np.where(full >= 1 << 31, full - (1 << 32), full)
            assert np.array_equal(dec, nbr[i, :act]), (name, k, i)
            n_mor += int(mor.sum()); n_dir += act
    if name == "tgv64_refined":
        assert n_wide > 0
    if name in ("sphere_d12", "d3q19_morton", "d2q9_morton") or (
            morton == "morton" and name in ("tgv64_refined", "d3q27_morton")):
        assert n_mor > 0.15 * n_dir, (name, n_mor, n_dir)


def test_morton_policy_rejects_bad_values():
    with pytest.raises(M.MLBMError):
        M.set_morton_policy(1.5, 6)
    with pytest.raises(M.MLBMError):
        M.set_morton_policy(0.5, 0)
    M.set_morton_policy()


def _morton_of(coords, d, L):
    m = np.zeros(coords.shape[1], dtype=np.uint64)
    for bit in range(L):
        for a in range(d):
            m |= ((coords[a].astype(np.uint64) >> np.uint64(bit)) & np.uint64(1)) << np.uint64(d * bit + a)
    return m


def test_every_header_symbol_is_exported():
    with open(os.path.join(ROOT, "include", "mlbm.h")) as fh:
        text = fh.read()
    names = set(re.findall(r"\b(mlbm_[a-z0-9_]+)\s*\(", text))
    assert len(names) > 20
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n


def _raw_create(stencil, level0, origin, extent, faces, leaves, solids=()):
    lib = _lib.lib()
    h = ctypes.c_void_p()
    o = np.asarray(origin, np.int32)
    e = np.asarray(extent, np.int32)
    f = np.asarray(faces, np.int32)
    lv = np.asarray(leaves, np.uint64)
    sv = np.asarray(solids, np.uint64)
    rc = lib.mlbm_plan_create(stencil, level0, o.ctypes.data_as(_lib._pi32),
                              e.ctypes.data_as(_lib._pi32), f.ctypes.data_as(_lib._pi32),
                              lv.ctypes.data_as(_lib._pu64), len(lv),
                              sv.ctypes.data_as(_lib._pu64) if len(sv) else None, len(sv),
                              ctypes.byref(h))
    if rc == 0:
        lib.mlbm_plan_destroy(h)
    return rc


def test_error_paths():
    spec = W.refined_box_mesh("D2Q9", 3, 2, 6)
    base = (0, 3, spec.box_origin, spec.box_extent, [0, 0, 0, 0], spec.leaf_ids)
    assert _raw_create(*base) == 0
    # hole: drop one leaf
    assert _raw_create(0, 3, (0, 0), (8, 8), [0] * 4, spec.leaf_ids[1:]) == _lib.E_MESH
    # overlap: add a parent of existing leaves
    from workloads.meshes import encode_tree_ids
    extra = encode_tree_ids(3, np.array([[2, 2]]))
    ids = np.concatenate([spec.leaf_ids, extra])
    assert _raw_create(0, 3, (0, 0), (8, 8), [0] * 4, ids) == _lib.E_MESH
    # bad stencil / unpaired periodic faces / box outside the root
    assert _raw_create(7, 3, (0, 0), (8, 8), [0] * 4, spec.leaf_ids) == _lib.E_ARG
    assert _raw_create(0, 3, (0, 0), (8, 8), [0, 1, 0, 0], spec.leaf_ids) == _lib.E_ARG
    assert "pairs" in _lib.lib().mlbm_last_error().decode()
    assert _raw_create(0, 3, (0, 0), (16, 8), [0] * 4, spec.leaf_ids) == _lib.E_ARG
    # refinement touching a coarser level two steps away (no nesting buffer)
    tight = W.refined_box_mesh("D2Q9", 4, 4, 12, extra_levels=[(8, 16)])
    rc = _raw_create(0, 4, tight.box_origin, tight.box_extent, [0] * 4, tight.leaf_ids)
    assert rc == _lib.E_MESH
    with pytest.raises(M.MLBMError):
        M.Plan("D2Q9", 4, tight.box_origin, tight.box_extent, ["periodic"] * 4,
               tight.leaf_ids)


def test_oracle_rejects_the_same_meshes():
    tight = W.refined_box_mesh("D2Q9", 4, 4, 12, extra_levels=[(8, 16)])
    with pytest.raises(omesh.MeshError):
        omesh.build(tight)


# ------------------------------------------------ wall fractions ----------
def _sphere_small(stencil="D3Q19"):
    return W.sphere_channel_mesh(8, 2, l0_per_d=4, length=(-2.0, 3.0), half_width=2.0,
                                 boxes_in_d=((-1.0, 1.5, 1.0),), stencil=stencil)


@pytest.mark.parametrize("stencil", ["D3Q19", "D3Q27"])
def test_wall_tables_match_oracle(stencil):
    """Links with a wall fraction: element, pull direction, second node and
    fraction equal the oracle's links (same treeIDs, bit-exact), sorted by
    element then direction."""
    from oracle.solver import wall_links
    spec = _sphere_small(stencil)
    om = omesh.build(spec)
    c_lib, _ = M.lattice(stencil)
    perm = [int(np.where((om.lattice.c == c_lib[i]).all(1))[0][0]) for i in range(len(c_lib))]
    ids, dirs, q = W.sphere_wall_links(spec, c_lib)
    plan = M.Plan.from_spec(spec)
    plan.set_walls(ids, dirs, q)
    ow = wall_links(om, *W.sphere_wall_links(spec, om.lattice.c))
    for k in range(plan.n_levels):
        L = plan.level0 + k
        n_w = plan.info[k]["n_wall"]
        if L not in ow:
            assert n_w == 0
            continue
        wt = plan.export(k, "wall")
        wq = plan.export(k, "wall_q")
        assert len(wt) == n_w == len(ow[L][0])
        gt = plan.export(k, "treeid")
        ot = om.lev(L).tid
        # library links as (treeID, oracle direction into the solid, q, treeID of x2)
        opp = lambda i: (i + 1) if i & 1 else (i - 1)
        mine = sorted((int(gt[x]), perm[opp(int(j))], float(qq), int(gt[x2]) if x2 >= 0 else -1)
                      for (x, j, x2, _), qq in zip(wt, wq))
        x, i, qo, x2 = ow[L]
        theirs = sorted((int(ot[a]), int(b), float(c), int(ot[e]) if e >= 0 else -1)
                        for a, b, c, e in zip(x, i, qo, x2))
        assert mine == theirs
        key = wt[:, 0].astype(np.int64) * 64 + wt[:, 1]
        assert (np.diff(key) > 0).all()


def test_set_walls_rejects_bad_links():
    spec = _sphere_small()
    c_lib, _ = M.lattice("D3Q19")
    ids, dirs, q = W.sphere_wall_links(spec, c_lib)
    plan = M.Plan.from_spec(spec)
    plan.set_walls(ids, dirs, q)
    n0 = sum(i["n_wall"] for i in plan.info)
    assert n0 == len(ids)

    def code(ids_, dirs_, q_):
        with pytest.raises(M.MLBMError) as e:
            plan.set_walls(ids_, dirs_, q_)
        return e.value.code
    bad_q = q.copy()
    bad_q[3] = 1.5
    assert code(ids, dirs, bad_q) == _lib.E_ARG
    bad_q[3] = np.nan
    assert code(ids, dirs, bad_q) == _lib.E_ARG
    bad_d = dirs.copy()
    bad_d[0] = len(c_lib)
    assert code(ids, bad_d, q) == _lib.E_ARG
    assert code(np.concatenate([ids, ids[:1]]), np.concatenate([dirs, dirs[:1]]),
                np.concatenate([q, q[:1]])) == _lib.E_ARG
    # a direction whose neighbour is fluid
    opp = (dirs[0] + 1) if dirs[0] & 1 else (dirs[0] - 1)
    assert code(ids[:1], np.array([opp], np.int32), q[:1]) == _lib.E_MESH
    # a solid cell is no fluid leaf
    assert code(spec.solid_ids[:1], dirs[:1], q[:1]) == _lib.E_MESH
    # failures leave the previous set in place; n = 0 clears it
    assert sum(i["n_wall"] for i in plan.info) == n0
    plan.set_walls([], [], [])
    assert sum(i["n_wall"] for i in plan.info) == 0
