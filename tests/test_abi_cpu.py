"""C-ABI library checks that need no GPU: it loads, exports every declared entry point,
the host tree builder matches the oracle's tree exactly, and argument validation."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle.tree import build_tree as oracle_tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "rs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rs_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1110_3105_amd as rs
    lib = ctypes.CDLL(rs.LIB_PATH)
    declared = _declared_symbols()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(lib, name), name
    assert set(rs.EXPORTED) <= set(declared)


@pytest.mark.parametrize("mk,leaf", [(lambda: W.star_curve(4096), 64),
                                     (lambda: W.star_curve(65536), 64),
                                     (lambda: W.random_curve(3000, [0.03, 0.01, 0.02], [0.1, 2.0, 4.0]), 32),
                                     (lambda: W.fibonacci_sphere(20480), 128),
                                     (lambda: W.ellipse(777), 16)])
def test_host_tree_matches_oracle_tree(mk, leaf):
    import paper_1110_3105_amd as rs
    g = mk()
    t = rs.build_tree(g.points, leaf)
    e = t.export()
    o = oracle_tree(g.points, leaf)
    assert np.array_equal(e["perm"], o.perm)
    assert np.array_equal(e["depth"], o.depth)
    assert np.array_equal(e["parent"], o.parent)
    assert np.array_equal(e["begin"], o.begin) and np.array_equal(e["end"], o.end)
    assert np.array_equal(e["center"], o.center) and np.array_equal(e["side"], o.side)


def test_host_tree_adaptive_cases_match_oracle_tree():
    """Boxes that stop splitting above the top levels built in one pass (a dense cluster
    with sparse outliers, a few points, collinear points, 3D clusters) keep the point
    order of splitting level by level: the oracle's tree, array for array."""
    import paper_1110_3105_amd as rs
    rng = np.random.default_rng(11)
    cases = [
        (np.concatenate([rng.normal(0.0, 1e-3, (3000, 2)), rng.random((40, 2))]), 8),
        (rng.random((7, 2)), 2),
        (np.stack([np.linspace(0.0, 1.0, 900), np.zeros(900)], axis=1), 10),
        (np.concatenate([rng.normal(0.0, 1e-2, (2000, 3)), 4.0 * rng.random((30, 3))]), 16),
        (np.repeat(rng.random((20, 2)), 30, axis=0), 8),
    ]
    for pts, leaf in cases:
        pts = np.ascontiguousarray(pts)
        e = rs.build_tree(pts, leaf).export()
        o = oracle_tree(pts, leaf)
        assert np.array_equal(e["perm"], o.perm)
        assert np.array_equal(e["depth"], o.depth) and np.array_equal(e["parent"], o.parent)
        assert np.array_equal(e["begin"], o.begin) and np.array_equal(e["end"], o.end)
        assert np.array_equal(e["center"], o.center) and np.array_equal(e["side"], o.side)


def test_tree_argument_errors():
    import paper_1110_3105_amd as rs
    with pytest.raises(rs.RSError) as ei:
        rs.build_tree(np.zeros((0, 2)), 8)
    assert ei.value.code == 1
    bad = np.array([[0.0, 1.0], [np.nan, 2.0]])
    with pytest.raises(rs.RSError):
        rs.build_tree(bad, 8)
    with pytest.raises(rs.RSError):
        rs.build_tree(np.zeros((5, 2)), 0)


def test_factor_argument_validation_before_device_use():
    import paper_1110_3105_amd as rs
    g = W.star_curve(256)
    t = rs.build_tree(g.points, 32)
    cases = [
        dict(kind="lap2d_dl"),                                   # no normals / curvature
        dict(kind="lap3d_sl"),                                   # dimension mismatch
        dict(kind="lap2d_sl", eps=-1.0),
        dict(kind="lap2d_sl", proxy_points=2),
        dict(kind="lap2d_sl", proxy_ratio=0.5),
        dict(kind="lap2d_sl", weights=-g.weights),
        dict(kind="lap2d_sl", points=g.points[::-1].copy()),      # not the tree's points
    ]
    for c in cases:
        args = dict(kind="lap2d_sl", points=g.points, weights=g.weights, eps=1e-9)
        args.update(c)
        with pytest.raises(rs.RSError) as ei:
            rs.factor(args["kind"], t, args["points"], args["weights"], args["eps"],
                      proxy_points=args.get("proxy_points", 64),
                      proxy_ratio=args.get("proxy_ratio", 1.5))
        assert ei.value.code == 1, c
    # per-point checks run over blocks of 8192 points on the host pool: a bad entry in
    # any block (the ragged last one included) is found, and the first failed check in
    # a fixed order is the one reported
    gl = W.star_curve(20000)
    tl = rs.build_tree(gl.points, 64)
    pts_nan = gl.points.copy()
    pts_nan[-1, 1] = np.nan
    w_neg = gl.weights.copy()
    w_neg[9000] = -1.0
    w_nan = gl.weights.copy()
    w_nan[17000] = np.nan
    moved = gl.points.copy()
    moved[16500, 0] += 1e-12
    for pts, w, msg in [(pts_nan, gl.weights, "non-finite points or weights"),
                        (gl.points, w_neg, "weights must be positive"),
                        (gl.points, w_nan, "non-finite points or weights"),
                        (moved, gl.weights, "points differ from the tree's points"),
                        (moved, w_neg, "weights must be positive")]:
        with pytest.raises(rs.RSError) as ei:
            rs.factor("lap2d_sl", tl, pts, w, 1e-9)
        assert ei.value.code == 1 and msg in str(ei.value), (msg, str(ei.value))
    helm = [dict(),                                            # no normals / curvature
            dict(normals=g.normals, curvature=g.curvature),     # wavenumber 0
            dict(normals=g.normals, curvature=g.curvature, wavenumber=float("nan")),
            dict(normals=g.normals, curvature=g.curvature, wavenumber=10.0, eta=float("inf"))]
    for c in helm:
        with pytest.raises(rs.RSError) as ei:
            rs.factor("helm2d_cfie", t, g.points, g.weights, 1e-9, **c)
        assert ei.value.code == 1, c


def test_tree_builds_from_concurrent_threads():
    # the host worker pool is shared by every thread that builds trees or plans levels;
    # concurrent callers must each get their own complete, correct result
    import threading
    import paper_1110_3105_amd as rs
    geoms = [W.star_curve(16384), W.random_curve(9000, [0.03, 0.01], [0.2, 1.3]),
             W.fibonacci_sphere(8000), W.ellipse(12000)]
    leaf = [64, 48, 128, 64]
    ref = [rs.build_tree(g.points, lf).export() for g, lf in zip(geoms, leaf)]
    errors = []

    def work(i):
        try:
            for _ in range(6):
                e = rs.build_tree(geoms[i].points, leaf[i]).export()
                for key in ("perm", "begin", "end", "parent", "depth"):
                    if not np.array_equal(e[key], ref[i][key]):
                        errors.append((i, key))
        except Exception as exc:          # pragma: no cover
            errors.append((i, repr(exc)))

    threads = [threading.Thread(target=work, args=(i % 4,)) for i in range(8)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors


def test_factor_estimate_rank_model():
    """rs_factor_estimate (host only): the footprint grows with N and with the decades of
    eps, complex kernels need more than real ones, and the resident part stays below the
    slots of every box at an active set of 128 (the largest ranks of this curve are below
    64, so no box of the model comes near it)."""
    import paper_1110_3105_amd as rs
    est = {}
    for n in (4096, 16384, 65536):
        g = W.star_curve(n)
        t = rs.build_tree(g.points, 64)
        for eps in (1e-6, 1e-9, 1e-12):
            est[n, eps] = rs.factor_estimate("lap2d_sl", t, eps)
        e = est[n, 1e-9]
        nb = t.info()[0]
        assert e["resident"] <= 8 * nb * (5 * 128 * 128 // 4 + 128 + 8)
        assert e["transient"] >= 64 << 20
        ec = rs.factor_estimate("helm2d_cfie", t, 1e-9, wavenumber=20.0)
        assert ec["resident"] > e["resident"]
    for n in (4096, 16384, 65536):
        assert est[n, 1e-6]["resident"] < est[n, 1e-9]["resident"] < est[n, 1e-12]["resident"]
    for eps in (1e-6, 1e-9, 1e-12):
        assert est[4096, eps]["resident"] < est[16384, eps]["resident"] < est[65536, eps]["resident"]
