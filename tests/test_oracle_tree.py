"""Pins of the oracle's tree (CPU): a hand-derived example and structural invariants."""
import numpy as np
import pytest

import workloads as W
from oracle.tree import build_tree


def test_hand_derived_quadtree():
    # Six points, leaf size 2.  Bounding box [0,4]x[0,2]: centre (2,1), side 4.
    # Codes (bit0: x >= 2, bit1: y >= 1):
    #   p0 (0.5,0.5)->0  p1 (3,0.2)->1  p2 (1,1.5)->2  p3 (0,0)->0  p4 (4,2)->3
    #   p5 (0.9,0.9)->0
    # Root children in code order: c0 {p0,p3,p5} (centre (1,0), side 2),
    # c1 {p1} (3,0), c2 {p2} (1,2), c3 {p4} (3,2).  c0 has 3 > 2 points: split at (1,0)
    # with side 1 -> codes: p0 (0.5,0.5): x<1,y>=0 -> 2; p3 (0,0) -> 2; p5 (0.9,0.9) -> 2:
    # all in child code 2 (centre (0.5,0.5), side 1), which splits
    # again at (0.5,0.5): p0 -> 3, p3 (0,0) -> 0, p5 -> 3, giving leaves {p3} and {p0,p5}.
    pts = np.array([[0.5, 0.5], [3, 0.2], [1, 1.5], [0.0, 0.0], [4.0, 2.0], [0.9, 0.9]])
    t = build_tree(pts, 2)
    assert t.nbox == 8
    assert list(t.depth) == [0, 1, 1, 1, 1, 2, 3, 3]
    assert list(t.parent) == [-1, 0, 0, 0, 0, 1, 5, 5]
    assert list(t.perm) == [3, 0, 5, 1, 2, 4]
    assert list(zip(t.begin, t.end)) == [(0, 6), (0, 3), (3, 4), (4, 5), (5, 6), (0, 3),
                                         (0, 1), (1, 3)]
    assert np.allclose(t.center[1], [1, 0]) and t.side[1] == 2.0
    assert np.allclose(t.center[5], [0.5, 0.5]) and t.side[5] == 1.0
    assert np.allclose(t.center[7], [0.75, 0.75]) and t.side[7] == 0.5


@pytest.mark.parametrize("maker,leaf", [(lambda: W.star_curve(4096), 64),
                                        (lambda: W.star_curve(1000), 16),
                                        (lambda: W.fibonacci_sphere(3000), 128)])
def test_tree_invariants(maker, leaf):
    g = maker()
    t = build_tree(g.points, leaf)
    assert sorted(t.perm.tolist()) == list(range(g.n))
    pts = g.points[t.perm]
    for b in range(t.nbox):
        lo, hi = t.begin[b], t.end[b]
        assert hi > lo                                   # empty boxes are dropped
        half = t.side[b] * 0.5
        inside = np.abs(pts[lo:hi] - t.center[b]) <= half + 1e-15 * t.side[0]
        assert inside.all()
        ch = t.children[b]
        if ch:
            assert t.end[b] - t.begin[b] > leaf
            assert t.begin[ch[0]] == lo and t.end[ch[-1]] == hi
            for a, c in zip(ch[:-1], ch[1:]):
                assert t.end[a] == t.begin[c]
            for c in ch:
                assert t.depth[c] == t.depth[b] + 1 and t.parent[c] == b
                assert t.side[c] == t.side[b] * 0.5
        else:
            assert hi - lo <= leaf
    # breadth-first numbering: depths non-decreasing
    assert np.all(np.diff(t.depth) >= 0)


def test_tree_stable_order_inside_leaf():
    g = W.star_curve(2048)
    t = build_tree(g.points, 64)
    for b in range(t.nbox):
        if not t.children[b]:
            seg = t.perm[t.begin[b]:t.end[b]]
            # within a leaf, caller order is preserved except for the wrap at index 0
            d = np.diff(seg)
            assert np.sum(d < 0) <= 1


def test_single_box_tree():
    g = W.star_curve(50)
    t = build_tree(g.points, 64)
    assert t.nbox == 1 and t.maxdepth == 0 and list(t.perm) == list(range(50))
