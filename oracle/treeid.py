"""treeID decoding, Z-curve order and workload weights (Sec. 3.1).

Reading taken (the paper only draws the 2D case): the root is id 0 at
level 0; children of element t are 2^d*t+1 ... 2^d*t+2^d; so the first id
of level L is sum_{k<L} 2^(d k); inside a level the offset is the Morton
code of the integer coordinates with the x bit least significant, then y,
then z.  The 2D figure of Sec. 3.1 fixes this numbering exactly.
"""
from __future__ import annotations

import numpy as np


def first_id(level: int, d: int) -> int:
    total = 0
    for k in range(level):
        total += 1 << (d * k)
    return total


def level_of(tid: int, d: int) -> int:
    level = 0
    while first_id(level + 1, d) <= tid:
        level += 1
    return level


def morton(coords: np.ndarray, bits: int) -> np.ndarray:
    """Morton code, x bit lowest; coords (n, d) non-negative ints."""
    coords = np.asarray(coords, dtype=np.int64)
    n, d = coords.shape
    out = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        for a in range(d):
            out |= ((coords[:, a] >> b) & 1) << (d * b + a)
    return out


def demorton(code: np.ndarray, d: int, bits: int) -> np.ndarray:
    code = np.asarray(code, dtype=np.int64)
    out = np.zeros((len(code), d), dtype=np.int64)
    for b in range(bits):
        for a in range(d):
            out[:, a] |= ((code >> (d * b + a)) & 1) << b
    return out


def decode(tids, d: int):
    """treeIDs -> (levels (n,), coords (n, d)) by the numbering above."""
    t64 = np.asarray(tids, dtype=np.uint64).reshape(-1)
    n = len(t64)
    # level boundaries up to 2^63
    firsts = []
    L = 0
    while True:
        f = first_id(L, d)
        if f >= (1 << 63):
            break
        firsts.append(f)
        L += 1
    firsts_arr = np.array(firsts, dtype=np.uint64)
    levels = np.searchsorted(firsts_arr, t64, side="right").astype(np.int64) - 1
    offsets = (t64 - firsts_arr[levels]).astype(np.int64)
    coords = np.zeros((n, d), dtype=np.int64)
    for lev in np.unique(levels):
        m = levels == lev
        coords[m] = demorton(offsets[m], d, int(lev))
    return levels, coords


def encode(level: int, coords: np.ndarray) -> np.ndarray:
    coords = np.asarray(coords, dtype=np.int64)
    d = coords.shape[1]
    return (np.uint64(first_id(level, d))
            + morton(coords, level).astype(np.uint64))


def sfc_order(tids, d: int) -> np.ndarray:
    """Permutation sorting mixed-level leaves along the Z curve: each leaf is
    placed by the Morton code of its first descendant on the finest level
    present (leaves never overlap, so this key is unique)."""
    levels, coords = decode(tids, d)
    lmax = int(levels.max())
    fine = coords << (lmax - levels)[:, None]
    key = morton(fine, lmax)
    return np.argsort(key, kind="stable")


def weights(levels: np.ndarray) -> np.ndarray:
    """Eq. weight: w_i = 2^(L_i - L_min)."""
    levels = np.asarray(levels, dtype=np.int64)
    return (1 << (levels - levels.min())).astype(np.int64)


def partition(tids, d: int, nproc: int):
    """Weight-based split of the Z-ordered list (Sec. 3.1): element i goes to
    process ceil(W_i / W_avg) where W is the cumulative weight.  Returns the
    sorted ids, weights, cumulative weights and 1-based process numbers."""
    order = sfc_order(tids, d)
    sorted_ids = np.asarray(tids, dtype=np.uint64)[order]
    levels, _ = decode(sorted_ids, d)
    w = weights(levels)
    W = np.cumsum(w)
    w_avg = W[-1] / nproc
    proc = np.ceil(W / w_avg).astype(np.int64)
    return sorted_ids, w, W, proc
