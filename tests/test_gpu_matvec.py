"""Compressed forward operator (rs_matvec) on the MI355X against the oracle.

Y = A_eps X by the telescoping representation of Section 3.3 (upward interpolation R,
the root block, downward interpolation L plus each level's diagonal blocks), with the
handle's own skeletons and interpolation matrices.  Checked against:

* the oracle's compressed_matvec on the oracle's factorization (the same skeletons on
  untied boxes, hence the same A_eps up to rounding): 10 eps in the normwise form
  |y - y_oracle| <= 10 eps |A|_2 |x| (for the first-kind kernels |A x| can be far
  below |A| |x|, and rounding in T moves A_eps by eps-sized amounts in directions the
  compression does not resolve);
* the dense matrix: A_eps agrees with A to the compression precision in the same
  normwise form (Section 5's estimate for the compressed matrix);
* eps = 0 (no compression): A_eps = A to rounding;
* the solve: A_eps (A_eps^{-1} b) = b to rounding, an O(N) residual at full size.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Problem, dense
from oracle import factor as ofactor
from oracle.embed import compressed_matvec
from parity_util import compare_skeletons, identical_skeletons, to_device

pytestmark = pytest.mark.gpu


def _setup(rs, kind, g, eps, leaf, npx, k=None):
    t = rs.build_tree(g.points, leaf)
    if kind == "lap2d_dl":
        p = Problem(kind, g.points, g.weights, g.normals, g.curvature, identity=-0.5)
        h = rs.factor(kind, t, g.points, g.weights, eps, normals=g.normals,
                      curvature=g.curvature, identity=-0.5, proxy_points=npx)
    elif kind == "helm2d_cfie":
        p = Problem(kind, g.points, g.weights, g.normals, g.curvature, identity=0.5,
                    wavenumber=k, eta=k)
        h = rs.factor(kind, t, g.points, g.weights, eps, normals=g.normals,
                      curvature=g.curvature, identity=0.5, proxy_points=npx,
                      wavenumber=k, eta=k)
    elif kind == "helm3d_sl":
        p = Problem(kind, g.points, g.weights, wavenumber=k)
        h = rs.factor(kind, t, g.points, g.weights, eps, proxy_points=npx, wavenumber=k)
    else:
        p = Problem(kind, g.points, g.weights, identity=0.0)
        h = rs.factor(kind, t, g.points, g.weights, eps, identity=0.0, proxy_points=npx)
    return p, h


def _mv(h, x):
    import torch
    X = to_device(x, h.dtype)
    Y = h.matvec(X)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


CASES = [
    ("lap2d_dl", lambda: W.star_curve(4096), 1e-9, 64, 64, None),
    ("lap2d_sl", lambda: W.star_curve(3000), 1e-6, 48, 64, None),
    ("lap3d_sl", lambda: W.fibonacci_sphere(2048), 1e-6, 128, 256, None),
    ("helm2d_cfie", lambda: W.star_curve(2048), 1e-9, 64, 64, 10.0),
    ("helm3d_sl", lambda: W.fibonacci_sphere(2048), 1e-6, 128, 256, 3.18),
]


@pytest.mark.parametrize("kind,mk,eps,leaf,npx,wl", CASES)
def test_matvec_matches_oracle(gpu_lib, kind, mk, eps, leaf, npx, wl):
    rs = gpu_lib
    g = mk()
    k = W.helmholtz_wavenumber(g, wl) if wl else None
    p, h = _setup(rs, kind, g, eps, leaf, npx, k)
    F = ofactor(p, eps, leaf, npx)
    _, tied = compare_skeletons(h, F)
    same = identical_skeletons(h, F)
    cplx = kind in ("helm2d_cfie", "helm3d_sl")
    A = dense.matrix(p)
    a2 = np.linalg.norm(A, 2)
    for nrhs in (1, 3, 17):
        x = W.gaussian_rhs(g.n, nrhs, 40 + nrhs, cplx)
        y = _mv(h, x)
        yo = compressed_matvec(F, x)
        ya = A @ x
        for j in range(nrhs):
            scale = a2 * np.linalg.norm(x[:, j])
            if same:
                assert np.linalg.norm(y[:, j] - yo[:, j]) <= 10 * eps * scale, (nrhs, j)
            assert np.linalg.norm(y[:, j] - ya[:, j]) <= 10 * eps * scale, (nrhs, j)


@pytest.mark.parametrize("n,leaf", [(700, 32), (50, 64)])
def test_matvec_eps_zero_is_dense(gpu_lib, n, leaf):
    rs = gpu_lib
    g = W.star_curve(n)
    p, h = _setup(rs, "lap2d_sl", g, 0.0, leaf, 64)
    x = W.gaussian_rhs(n, 5, 7)
    y = _mv(h, x)
    ya = dense.matrix(p) @ x
    assert np.linalg.norm(y - ya) / np.linalg.norm(ya) <= 1e-13


def test_matvec_inverts_solve(gpu_lib):
    """A_eps applied to the solve's output returns the right-hand side."""
    import torch
    rs = gpu_lib
    g = W.star_curve(8192)
    p, h = _setup(rs, "lap2d_dl", g, 1e-9, 64, 64)
    b = W.gaussian_rhs(g.n, 20, 3)
    B = to_device(b)
    h.solve(B)
    Y = h.matvec(B)
    torch.cuda.synchronize()
    y = Y.cpu().numpy()
    assert np.linalg.norm(y - b) / np.linalg.norm(b) <= 1e-12


def test_matvec_full_size_parity(gpu_lib):
    """The benchmark workload (star, N = 65536, log single layer, eps = 1e-9): the
    solve's residual against A_eps over all N rows; A_eps applied to smooth densities
    (|A x| ~ |A| |x|) against the oracle's compressed operator over all rows, and
    against the exact matrix on sampled rows, where the device may be off by no more
    than the oracle's own compression error plus 10 eps (at this size the compressed
    operator differs from A by about 4e-8 relative, on both sides)."""
    import torch
    rs = gpu_lib
    n, eps = 65536, 1e-9
    g = W.star_curve(n)
    p, h = _setup(rs, "lap2d_sl", g, eps, 64, 64)
    b = W.gaussian_rhs(n, 4, 1)
    B = to_device(b)
    h.solve(B)
    Y = h.matvec(B)
    torch.cuda.synchronize()
    y = Y.cpu().numpy()
    # first kind (kappa ~ 4e4 here): the residual of the computed solution against the
    # operator it inverts is rounding times the conditioning
    assert np.linalg.norm(y - b) / np.linalg.norm(b) <= 1e-9
    F = ofactor(p, eps, 64, 64)
    same = identical_skeletons(h, F)
    th = 2.0 * np.pi * np.arange(n) / n
    xs = np.stack([1.0 + 0.0 * th, np.cos(3 * th), np.sin(7 * th) + 0.5 * np.cos(th)], axis=1)
    ys = _mv(h, xs)
    yo = compressed_matvec(F, xs)
    rows = np.random.default_rng(5).choice(n, 64, replace=False)
    ya = dense.matvec_rows(p, rows, xs)
    for j in range(xs.shape[1]):
        if same:
            assert np.linalg.norm(ys[:, j] - yo[:, j]) <= 10 * eps * np.linalg.norm(yo[:, j]), j
        err_gpu = np.linalg.norm(ys[rows, j] - ya[:, j]) / np.linalg.norm(ya[:, j])
        err_or = np.linalg.norm(yo[rows, j] - ya[:, j]) / np.linalg.norm(ya[:, j])
        assert err_gpu <= err_or + 10 * eps, (j, err_gpu, err_or)
