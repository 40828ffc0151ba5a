"""Quadtree / octree over the nodes with contiguous index ranges (oracle).

Follows Section 2.1 (each node of the index tree is a contiguous subsequence of the
reordered index vector; children concatenate to the parent) and the tree rule stated
for the experiments in Section 6 (uniform subdivision until blocks are O(1),
truncating empty boxes).  Concrete reading used here:

* root = the bounding square / cube of the nodes: centre (lo + hi) * 0.5 per axis,
  side = max over axes of (hi - lo);
* a box is split iff it holds more than ``leaf_size`` nodes (and its depth is below
  ``MAX_DEPTH`` and its side is positive);
* child code = sum_a [x_a >= c_a] << a; children are visited in increasing code,
  empty children are dropped, and the order of nodes inside a child is the order
  they had in the parent (stable);
* child centre c_a +/- side * 0.25, child side = side * 0.5 (exact in binary64);
* boxes are numbered breadth-first (depth by depth, in tree order inside a depth).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

MAX_DEPTH = 40


@dataclass
class Tree:
    dim: int
    n: int
    leaf_size: int
    perm: np.ndarray            # tree position i holds caller node perm[i]
    center: np.ndarray          # (nbox, dim)
    side: np.ndarray            # (nbox,)
    depth: np.ndarray           # (nbox,)
    parent: np.ndarray          # (nbox,), -1 for the root
    begin: np.ndarray           # (nbox,) first tree position
    end: np.ndarray             # (nbox,) one past the last tree position
    children: List[List[int]] = field(default_factory=list)

    @property
    def nbox(self) -> int:
        return int(self.side.shape[0])

    @property
    def maxdepth(self) -> int:
        return int(self.depth.max())

    def is_leaf(self, b: int) -> bool:
        return len(self.children[b]) == 0

    def boxes_at(self, d: int) -> List[int]:
        return [b for b in range(self.nbox) if self.depth[b] == d]

    @property
    def iperm(self) -> np.ndarray:
        ip = np.empty_like(self.perm)
        ip[self.perm] = np.arange(self.n)
        return ip


def build_tree(points: np.ndarray, leaf_size: int) -> Tree:
    pts = np.asarray(points, dtype=np.float64)
    n, dim = pts.shape
    if n < 1 or leaf_size < 1:
        raise ValueError("need at least one node and leaf_size >= 1")
    lo = pts.min(axis=0)
    hi = pts.max(axis=0)
    c0 = (lo + hi) * 0.5
    s0 = float(np.max(hi - lo))
    perm = np.arange(n, dtype=np.int64)

    center, side, depth, parent, begin, end, children = [], [], [], [], [], [], []

    def add(c, s, d, p, b, e):
        center.append(np.array(c, dtype=np.float64))
        side.append(s)
        depth.append(d)
        parent.append(p)
        begin.append(b)
        end.append(e)
        children.append([])
        return len(side) - 1

    add(c0, s0, 0, -1, 0, n)
    q = 0
    while q < len(side):          # breadth-first: boxes are appended in BFS order
        b, e = begin[q], end[q]
        if e - b > leaf_size and depth[q] < MAX_DEPTH and side[q] > 0.0:
            idx = perm[b:e].copy()
            c = center[q]
            code = np.zeros(e - b, dtype=np.int64)
            for a in range(dim):
                code |= (pts[idx, a] >= c[a]).astype(np.int64) << a
            off = b
            for cc in range(1 << dim):
                sel = idx[code == cc]
                if sel.size == 0:
                    continue
                perm[off:off + sel.size] = sel
                cc_center = [c[a] + side[q] * 0.25 if (cc >> a) & 1 else c[a] - side[q] * 0.25
                             for a in range(dim)]
                ch = add(cc_center, side[q] * 0.5, depth[q] + 1, q, off, off + sel.size)
                children[q].append(ch)
                off += sel.size
        q += 1

    return Tree(dim, n, leaf_size, perm, np.array(center), np.array(side),
                np.array(depth, dtype=np.int64), np.array(parent, dtype=np.int64),
                np.array(begin, dtype=np.int64), np.array(end, dtype=np.int64), children)
