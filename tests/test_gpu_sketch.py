"""Randomized ID (RS_ID_SKETCH) on the MI355X against the oracle's randomized ID.

Each box's block M is compressed through its row sketch Y = Omega M (Omega: random
signs from the SplitMix64 counter-based generator, reproduced exactly on both sides; ell
= min(m, n + oversample) rows).  With the same seed the device and the oracle sketch the
same blocks with the same signs, so they choose the same skeletons wherever no tie can
reach a box (ties judged on the sketch, with the rounding width of the original block's
row count); the solutions then agree to 10 eps, and every launch organisation gives
bitwise the same result.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Problem, dense
from oracle import factor as ofactor
from parity_util import compare_skeletons, identical_skeletons, to_device

pytestmark = pytest.mark.gpu

SEED, OVS = 20240613, 16


def _solve(h, b, mode="level"):
    import torch
    B = to_device(b, h.dtype)
    h.solve(B, launch_mode=mode)
    torch.cuda.synchronize()
    return B.cpu().numpy()


CASES = [
    ("lap2d_dl", lambda: W.star_curve(4096), 1e-9, 64, 64),
    ("lap3d_sl", lambda: W.fibonacci_sphere(2048), 1e-6, 128, 256),
    ("helm2d_cfie", lambda: W.star_curve(2048), 1e-9, 64, 64),
]


@pytest.mark.parametrize("kind,mk,eps,leaf,npx", CASES)
def test_sketch_parity_with_oracle(gpu_lib, kind, mk, eps, leaf, npx):
    rs = gpu_lib
    g = mk()
    extra, pk = {}, {}
    if kind == "lap2d_dl":
        extra = dict(normals=g.normals, curvature=g.curvature, identity=-0.5)
        pk = dict(normals=g.normals, curvature=g.curvature, identity=-0.5)
    elif kind == "helm2d_cfie":
        k = W.helmholtz_wavenumber(g, 8.0)
        extra = dict(normals=g.normals, curvature=g.curvature, identity=0.5, wavenumber=k, eta=k)
        pk = dict(normals=g.normals, curvature=g.curvature, identity=0.5, wavenumber=k, eta=k)
    p = Problem(kind, g.points, g.weights, **pk)
    F = ofactor(p, eps, leaf, npx, id_mode="sketch", sketch_seed=SEED, oversample=OVS)
    t = rs.build_tree(g.points, leaf)
    h = rs.factor(kind, t, g.points, g.weights, eps, proxy_points=npx, id_mode="sketch",
                  sketch_seed=SEED, oversample=OVS, **extra)
    compared, tied = compare_skeletons(h, F)
    same = identical_skeletons(h, F)
    assert compared >= 0.8 * len(F.records)
    cplx = kind == "helm2d_cfie"
    b = W.gaussian_rhs(g.n, 3, 17, complex_valued=cplx)
    x = _solve(h, b)
    xo = F.solve(b)
    if same:
        assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 10 * eps
    A = dense.matrix(p)
    res = np.linalg.norm(A @ x - b) / np.linalg.norm(b)
    reso = np.linalg.norm(A @ xo - b) / np.linalg.norm(b)
    assert res <= max(10 * eps, 2 * reso), (res, reso)
    # per-box launches: bitwise the same
    h2 = rs.factor(kind, t, g.points, g.weights, eps, proxy_points=npx, id_mode="sketch",
                   sketch_seed=SEED, oversample=OVS, launch_mode="per_box", **extra)
    assert np.array_equal(h2.box_skeletons()[0], h.box_skeletons()[0])
    assert np.array_equal(_solve(h2, b), x)


def test_sketch_seed_changes_compression(gpu_lib):
    rs = gpu_lib
    g = W.fibonacci_sphere(2048)
    t = rs.build_tree(g.points, 128)
    h1 = rs.factor("lap3d_sl", t, g.points, g.weights, 1e-6, proxy_points=256, id_mode="sketch",
                   sketch_seed=1)
    h2 = rs.factor("lap3d_sl", t, g.points, g.weights, 1e-6, proxy_points=256, id_mode="sketch",
                   sketch_seed=2)
    k1, s1 = h1.box_skeletons()
    k2, s2 = h2.box_skeletons()
    assert any(not np.array_equal(a, b) for a, b in zip(s1, s2))
    b = W.gaussian_rhs(g.n, 1, 3)
    x1, x2 = _solve(h1, b), _solve(h2, b)
    # two valid compressions: each solution is within 2 eps kappa of the exact one
    # (Section 5), so they are within twice that of each other
    kappa = np.linalg.cond(dense.matrix(Problem("lap3d_sl", g.points, g.weights)))
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) <= 4e-6 * kappa


def test_sketch_sphere_full_size_residual(gpu_lib):
    """The 3D configuration (unit sphere, N = 20480, eps = 1e-6, leaf 128, 512 proxies)
    compressed through sketches: the residual on sampled rows of the exact matrix stays
    within 10 eps of the right-hand side, as for the deterministic ID."""
    rs = gpu_lib
    n, eps = 20480, 1e-6
    g = W.fibonacci_sphere(n)
    t = rs.build_tree(g.points, 128)
    h = rs.factor("lap3d_sl", t, g.points, g.weights, eps, proxy_points=512, id_mode="sketch",
                  sketch_seed=SEED, oversample=OVS)
    b = W.gaussian_rhs(n, 2, 2)
    x = _solve(h, b)
    p = Problem("lap3d_sl", g.points, g.weights)
    rows = np.random.default_rng(1).choice(n, 48, replace=False)
    r = dense.matvec_rows(p, rows, x) - b[rows]
    for j in range(2):
        assert np.linalg.norm(r[:, j]) <= 10 * eps * np.linalg.norm(b[rows, j])
