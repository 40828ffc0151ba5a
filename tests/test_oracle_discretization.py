"""Pins of the oracle's matrix entries against closed forms (CPU).

These fix the kernels, the column weighting and the diagonal rules of oracle.green
independently of the oracle's own code: each expected value is a fact of potential
theory on a circle or sphere, not a re-evaluation of the same formula.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Problem, dense


def _sl2(g):
    return Problem("lap2d_sl", g.points, g.weights)


def _dl2(g, c=-0.5):
    return Problem("lap2d_dl", g.points, g.weights, g.normals, g.curvature, identity=c)


def _cfie(g, k, eta, c=0.5):
    return Problem("helm2d_cfie", g.points, g.weights, g.normals, g.curvature, identity=c,
                   wavenumber=k, eta=eta)


@pytest.mark.parametrize("n", [64, 333, 1024])
def test_unit_circle_double_layer_closed_form(n):
    # On the unit circle (x-y).nu_y / |x-y|^2 = -1/2 for every pair, so with the
    # curvature diagonal the interior equation matrix is -1/2 I - (1/2N) 1 1^T exactly.
    g = W.circle(n)
    A = dense.matrix(_dl2(g))
    expect = -0.5 * np.eye(n) - np.ones((n, n)) / (2 * n)
    assert np.abs(A - expect).max() < 1e-14


def test_double_layer_gauss_lemma_on_star():
    # Gauss: the double-layer potential of a unit density is -1/2 on the boundary.
    g = W.star_curve(1024)
    A = dense.matrix(_dl2(g, c=0.0))
    assert np.abs(A.sum(axis=1) + 0.5).max() < 1e-12


def test_double_layer_gauss_lemma_on_ellipse():
    g = W.ellipse(1024)
    A = dense.matrix(_dl2(g, c=0.0))
    assert np.abs(A.sum(axis=1) + 0.5).max() < 1e-12


def test_unit_circle_single_layer_constant_mode_exact():
    # The log single layer annihilates constants on the unit circle; the diagonal rule
    # is the one that makes the equispaced sum exact for that mode.
    for n in (100, 1024):
        A = dense.matrix(_sl2(W.circle(n)))
        assert np.abs(A @ np.ones(n)).max() < 1e-14


@pytest.mark.parametrize("m", [1, 2, 5, 10])
def test_unit_circle_single_layer_eigenvalues(m):
    # S[cos m t] = cos(m t) / (2m) on the unit circle; third-order convergence.
    errs = []
    for n in (256, 1024):
        A = dense.matrix(_sl2(W.circle(n)))
        t = 2 * np.pi * np.arange(n) / n
        v = np.cos(m * t)
        errs.append(np.abs(A @ v - v / (2 * m)).max())
    assert errs[1] < 1e-6
    assert errs[0] / errs[1] > 30.0          # ~ 4^3


def test_single_layer_sign_and_scale_off_circle():
    # On a circle of radius R the constant mode has eigenvalue -R log R (log kernel).
    R = 0.5
    n = 512
    A = dense.matrix(_sl2(W.circle(n, radius=R)))
    assert np.abs(A @ np.ones(n) - (-R * np.log(R))).max() < 1e-12


def test_sphere_single_layer_constant_and_dipole():
    # On the unit sphere S[1] = 1 and S[Y_1] = Y_1 / 3; first-order in the mesh size
    # with the flat-disc diagonal.
    errs1, errsy = [], []
    for n in (512, 2048):
        g = W.fibonacci_sphere(n)
        A = dense.matrix(Problem("lap3d_sl", g.points, g.weights))
        z = g.points[:, 2]
        errs1.append(np.abs(A.sum(axis=1) - 1.0).max())
        errsy.append(np.abs(A @ z - z / 3.0).max())
    assert errs1[1] < 3e-3 and errsy[1] < 3e-3
    assert errs1[0] / errs1[1] > 1.8 and errsy[0] / errsy[1] > 1.8


def test_nystrom_weights_on_columns():
    # A_ij = K(x_i, x_j) w_j: scaling one weight scales exactly one column.
    g = W.star_curve(64)
    p = _sl2(g)
    A = dense.matrix(p)
    w2 = g.weights.copy()
    w2[7] *= 3.0
    A2 = dense.matrix(Problem("lap2d_sl", g.points, w2))
    off = np.ones(64, dtype=bool)
    off[7] = False
    assert np.allclose(A2[off, 7], 3.0 * A[off, 7], rtol=1e-15, atol=0)
    assert np.array_equal(np.delete(A2, 7, axis=1), np.delete(A, 7, axis=1))


def test_curve_generators_closed_forms():
    # Circle of radius 1: weights 2 pi / N, curvature 1, normal = position.
    g = W.circle(37)
    assert np.allclose(g.weights, 2 * np.pi / 37, rtol=1e-15)
    assert np.allclose(g.curvature, 1.0, rtol=1e-14)
    assert np.allclose(g.normals, g.points, atol=1e-15)
    # Star: total length by the trapezoid rule converges spectrally; area via normals.
    s = W.star_curve(4096)
    area = 0.5 * np.sum(np.sum(s.points * s.normals, axis=1) * s.weights)
    assert abs(area - np.pi * (1 + 0.3 ** 2 / 2)) < 1e-12
    # Total curvature of a simple closed curve is 2 pi.
    assert abs(np.sum(s.curvature * s.weights) - 2 * np.pi) < 1e-10


@pytest.mark.parametrize("m", [0, 1, 3, 8])
def test_unit_circle_cfie_eigenvalues(m):
    # Graf's addition theorem on the unit circle: the Helmholtz single layer maps
    # e^{imt} to (i pi/2) J_m(k) H_m(k) e^{imt}, the double layer (principal value, outward
    # normal) to ((i pi k/2) J_m(k) H_m'(k) + 1/2) e^{imt}.  With A = c I + D - i eta S,
    # every Fourier mode is an eigenvector; the equispaced rule with the diagonal rule
    # converges to it at third order (m = 0 exercises the log(k/2) + gamma term).
    from scipy.special import h1vp, hankel1, jv
    k, eta, c = 10.0, 10.0, 0.5
    lam_s = 0.5j * np.pi * jv(m, k) * hankel1(m, k)
    lam_d = 0.5j * np.pi * k * jv(m, k) * h1vp(m, k) + 0.5
    lam = c + lam_d - 1j * eta * lam_s
    errs = []
    for n in (256, 1024):
        A = dense.matrix(_cfie(W.circle(n), k, eta, c))
        t = 2 * np.pi * np.arange(n) / n
        v = np.exp(1j * m * t)
        errs.append(np.abs(A @ v - lam * v).max())
    assert errs[1] < 2e-6
    assert errs[0] / errs[1] > 30          # ~ 4^3 for a quadrupled N


def test_cfie_diagonal_rule_sign_and_coupling():
    # The eta-part of the operator is -i eta S_k: with eta doubled and c = 0, D fixed,
    # A(eta2) - A(eta1) = -i (eta2 - eta1) S_k.  S_k's diagonal rule makes the unit
    # circle's constant mode exact to the quadrature order: S_k[1] = (i pi/2) J_0 H_0.
    from scipy.special import hankel1, jv
    k, n = 7.0, 1024
    g = W.circle(n)
    A1 = dense.matrix(_cfie(g, k, 1.0, 0.0))
    A2 = dense.matrix(_cfie(g, k, 3.0, 0.0))
    S = (A2 - A1) / (-2j)
    ones = np.ones(n)
    expect = 0.5j * np.pi * jv(0, k) * hankel1(0, k)
    assert np.abs(S @ ones - expect).max() < 1e-6
    # the real-valued Laplace single layer is the k -> 0 limit of S_k minus its constant
    S0 = dense.matrix(_sl2(g))
    ks = 1e-4
    Sk = (dense.matrix(_cfie(g, ks, 3.0, 0.0)) - dense.matrix(_cfie(g, ks, 1.0, 0.0))) / (-2j)
    const = 0.25j - (np.log(ks / 2) + 0.57721566490153286) / (2 * np.pi)
    W_ = np.tile(g.weights, (n, 1))
    assert np.abs(Sk - const * W_ - S0).max() < 1e-7


@pytest.mark.parametrize("kind,chunk", [("lap2d_sl", 1000), ("lap2d_sl", 701),
                                        ("lap2d_dl", 3000), ("lap2d_dl", 4096),
                                        ("helm2d_cfie", 512), ("helm2d_cfie", 999)])
def test_matvec_rows_equals_dense_rows(kind, chunk):
    # The chunked row matvec (used for residuals where A does not fit) against rows of the
    # assembled matrix, with chunk sizes that divide N, do not divide it, equal it and
    # exceed it.
    from oracle import dense
    n = 3000
    g = W.star_curve(n)
    if kind == "lap2d_sl":
        p = Problem(kind, g.points, g.weights)
    elif kind == "lap2d_dl":
        p = Problem(kind, g.points, g.weights, g.normals, g.curvature, identity=-0.5)
    else:
        k = W.helmholtz_wavenumber(g, 4.0)
        p = Problem(kind, g.points, g.weights, g.normals, g.curvature, identity=0.5,
                    wavenumber=k, eta=k)
    A = dense.matrix(p)
    rng = np.random.default_rng(4)
    rows = np.sort(rng.choice(n, 37, replace=False))
    rows = np.concatenate([rows, [0, n - 1]])      # first and last rows, unsorted tail
    for x in (rng.standard_normal(n), rng.standard_normal((n, 3))):
        if kind == "helm2d_cfie":
            x = x + 1j * rng.standard_normal(x.shape)
        ref = A[rows] @ x
        got = dense.matvec_rows(p, rows, x, chunk=chunk)
        assert got.shape == ref.shape
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(A[rows]).sum(axis=1).max() * np.abs(x).max()


def test_sphere_helmholtz_single_layer_eigenvalues():
    # On the unit sphere the Helmholtz single layer maps the spherical harmonic Y_n to
    # i k j_n(k) h_n(k) Y_n (h_n = j_n + i y_n, the outgoing spherical Hankel function):
    # S_k[1] = i k j_0 h_0 = sin(k) e^{ik} / k and S_k[z] = i k j_1 h_1 z.  The flat-disc
    # diagonal rule converges at first order in the mesh size, as for the Laplace kernel.
    from scipy.special import spherical_jn, spherical_yn
    k = 2 * np.pi * 3.18 / 2.0          # 3.18 wavelengths across the unit sphere
    lam = [1j * k * spherical_jn(nn, k) * (spherical_jn(nn, k) + 1j * spherical_yn(nn, k))
           for nn in (0, 1)]
    assert abs(lam[0] - np.sin(k) * np.exp(1j * k) / k) < 1e-14
    errs0, errs1 = [], []
    for n in (512, 2048):
        g = W.fibonacci_sphere(n)
        A = dense.matrix(Problem("helm3d_sl", g.points, g.weights, wavenumber=k))
        z = g.points[:, 2]
        errs0.append(np.abs(A @ np.ones(n) - lam[0]).max())
        errs1.append(np.abs(A @ z - lam[1] * z).max())
    assert errs0[1] < 1e-2 and errs1[1] < 1e-2
    assert errs0[0] / errs0[1] > 1.8 and errs1[0] / errs1[1] > 1.8


def test_helmholtz_3d_low_frequency_limit():
    # k -> 0: exp(ikr)/(4 pi r) -> 1/(4 pi r) entry by entry, off the diagonal and on it
    # ((e^{ikR} - 1)/(2ik) -> R/2), with an O(k) difference.
    g = W.fibonacci_sphere(300)
    A0 = dense.matrix(Problem("lap3d_sl", g.points, g.weights))
    for k in (1e-3, 1e-5):
        Ak = dense.matrix(Problem("helm3d_sl", g.points, g.weights, wavenumber=k))
        assert np.abs(Ak - A0).max() < 0.2 * k * np.abs(A0).max() + 1e-14
