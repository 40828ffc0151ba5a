"""Per-level records of a factorization (rs_query_levels) on the MI355X.

Each compressed level's record must add up the boxes of that depth (count, active DOFs
n, ranks k, largest active set and stored doubles of the Schur-form factors), the root's
record must be the root block, the levels must add up to the handle's totals, and the
device times must be positive and no larger than the whole factorization.  In a batched
factorization every problem keeps its own counts.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _check_levels(h, t):
    st = h.stats()
    lv = h.levels()
    tr = t.export()
    ks, _ = h.box_skeletons()
    assert lv[-1]["depth"] == 0 and all(a["depth"] > b["depth"] for a, b in zip(lv[:-2], lv[1:-1]))
    assert [e["depth"] for e in lv[:-1]] == list(range(st["maxdepth"], 0, -1))
    doubles = 0
    for e in lv[:-1]:
        boxes = [b for b in range(st["nbox"]) if tr["depth"][b] == e["depth"] and ks[b] >= 0]
        assert e["boxes"] == len(boxes)
        ns = [h.box_export(b)[0].size for b in boxes]
        assert e["n_total"] == sum(ns)
        assert e["max_n"] == max(ns)
        assert e["k_total"] == int(sum(ks[b] for b in boxes))
        assert e["max_m"] >= 0
        assert e["device_ms"] > 0 and e["plan_ms"] >= 0
        doubles += e["factor_doubles"]
    root = lv[-1]
    assert root["boxes"] == 1 and root["n_total"] == root["max_n"] == st["root_size"]
    assert root["device_ms"] > 0
    es = 2 if h.is_complex else 1
    assert root["factor_doubles"] == st["root_size"] ** 2 * es
    assert doubles + root["factor_doubles"] == st["factor_doubles"]
    assert sum(e["device_ms"] for e in lv) <= st["factor_ms"] * 1.01 + 0.05
    # the active DOFs of a level are the skeletons its children pass up plus the points
    # of its leaves; the root's are the skeletons of depth 1
    nchild = np.bincount(tr["parent"][tr["parent"] >= 0], minlength=st["nbox"])
    by_depth = {e["depth"]: e for e in lv}
    for e in lv[:-1] + [root]:
        d = e["depth"]
        leaf_pts = sum(int(tr["end"][b] - tr["begin"][b]) for b in range(st["nbox"])
                       if tr["depth"][b] == d and nchild[b] == 0)
        passed_up = by_depth[d + 1]["k_total"] if d + 1 in by_depth else 0
        assert e["n_total"] == passed_up + leaf_pts, d
    return lv


def test_levels_single_and_batched(gpu_lib):
    rs = gpu_lib
    g = W.star_curve(8192)
    t = rs.build_tree(g.points, 64)
    h = rs.factor("lap2d_sl", t, g.points, g.weights, 1e-9, proxy_points=64)
    lv = _check_levels(h, t)
    gs = W.fibonacci_sphere(6000)
    ts = rs.build_tree(gs.points, 128)
    k = W.helmholtz_wavenumber(gs, 2.0)
    hs = rs.factor("helm3d_sl", ts, gs.points, gs.weights, 1e-6, proxy_points=256,
                   wavenumber=k)
    _check_levels(hs, ts)
    # batched: the same counts per problem as the single factorizations
    gb = W.fibonacci_sphere(4000)
    tb = rs.build_tree(gb.points, 128)
    hb1 = rs.factor("lap3d_sl", tb, gb.points, gb.weights, 1e-6, proxy_points=256)
    lvb = _check_levels(hb1, tb)
    hb = rs.factor_batched([
        dict(kind="lap2d_sl", tree=t, points=g.points, weights=g.weights, eps=1e-9,
             proxy_points=64),
        dict(kind="lap3d_sl", tree=tb, points=gb.points, weights=gb.weights, eps=1e-6,
             proxy_points=256),
    ])
    keys = ("depth", "boxes", "n_total", "k_total", "max_n", "max_m", "factor_doubles")
    for (hh, tt), ref in zip(zip(hb, (t, tb)), (lv, lvb)):
        got = _check_levels(hh, tt)
        assert [tuple(e[q] for q in keys) for e in got] == [tuple(e[q] for q in keys) for e in ref]
