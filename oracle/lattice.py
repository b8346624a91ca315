"""DdQq velocity sets (Sec. 2.1).

The paper runs D2Q9 and D3Q27; this oracle provides those two and D3Q19.
Weights are the standard ones for which sum_i w_i = 1,
sum_i w_i c_ia c_ib = cs2 delta_ab and the fourth moment is isotropic with
cs2 = 1/3.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

CS2 = 1.0 / 3.0


@dataclass(frozen=True)
class Lattice:
    name: str
    d: int
    q: int
    c: np.ndarray      # (q, d) int64
    w: np.ndarray      # (q,) float64
    opp: np.ndarray    # (q,) int64

    def c_t(self, dtype=torch.float64) -> torch.Tensor:
        return torch.tensor(self.c, dtype=dtype)

    def w_t(self, dtype=torch.float64) -> torch.Tensor:
        return torch.tensor(self.w, dtype=dtype)


def _make(name: str, vecs, weights) -> Lattice:
    c = np.array(vecs, dtype=np.int64)
    w = np.array(weights, dtype=np.float64)
    opp = np.array([int(np.where((c == -c[i]).all(1))[0][0]) for i in range(len(c))])
    return Lattice(name, c.shape[1], c.shape[0], c, w, opp)


def d2q9() -> Lattice:
    vecs = [(0, 0)]
    wts = [4.0 / 9.0]
    for v in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
        vecs.append(v)
        wts.append(1.0 / 9.0)
    for v in [(1, 1), (-1, -1), (1, -1), (-1, 1)]:
        vecs.append(v)
        wts.append(1.0 / 36.0)
    return _make("D2Q9", vecs, wts)


def d3q19() -> Lattice:
    vecs = [(0, 0, 0)]
    wts = [1.0 / 3.0]
    for a in range(3):
        for s in (1, -1):
            v = [0, 0, 0]
            v[a] = s
            vecs.append(tuple(v))
            wts.append(1.0 / 18.0)
    for a, b in [(0, 1), (0, 2), (1, 2)]:
        for sa, sb in [(1, 1), (-1, -1), (1, -1), (-1, 1)]:
            v = [0, 0, 0]
            v[a], v[b] = sa, sb
            vecs.append(tuple(v))
            wts.append(1.0 / 36.0)
    return _make("D3Q19", vecs, wts)


def d3q27() -> Lattice:
    """Every c in {-1, 0, 1}^3: weight 8/27 at rest, 2/27 along an axis, 1/54
    across an edge (two non-zero components), 1/216 to a corner."""
    vecs, wts = [], []
    by_count = {0: 8.0 / 27.0, 1: 2.0 / 27.0, 2: 1.0 / 54.0, 3: 1.0 / 216.0}
    for v in np.ndindex(3, 3, 3):
        c = tuple(x - 1 for x in v)
        vecs.append(c)
        wts.append(by_count[sum(1 for x in c if x != 0)])
    return _make("D3Q27", vecs, wts)


def get(name: str) -> Lattice:
    return {"D2Q9": d2q9, "D3Q19": d3q19, "D3Q27": d3q27}[name]()
