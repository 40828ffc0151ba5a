"""End-to-end pins of the oracle's recursive skeletonization (CPU).

* eps = 0: no box compresses, so the method reduces to dense Gaussian elimination;
* brute force: the error bounds of Section 5 against a dense LU solve;
* the sparse-embedding formulation of Section 3.4 (sparse LU on the embedding) gives
  the same x as the telescoping inverse;
* the compressed forward operator reproduces b from x and approximates A to ~eps;
* the paper's Lambda = (R D^-1 L)^-1 equals the Schur complement of the transformed
  diagonal block, the form the device path computes;
* proxy compression is valid against the true far field;
* a physical check: interior Dirichlet data from an exterior point source.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Problem, dense, factor
from oracle.embed import compressed_matvec, embedding_solve
from oracle.green import block, kernel
from oracle.rs import compression_block, near_dofs


def dl_prob(g, c=-0.5):
    return Problem("lap2d_dl", g.points, g.weights, g.normals, g.curvature, identity=c)


def sl_prob(g):
    return Problem("lap2d_sl", g.points, g.weights)


def sph_prob(g):
    return Problem("lap3d_sl", g.points, g.weights)


def helm_prob(g, wavelengths=5.0):
    # exterior combined-field equation (1/2 I + D - i k S) sigma = f, k giving the stated
    # number of wavelengths across the domain's diameter
    k = W.helmholtz_wavenumber(g, wavelengths)
    return Problem("helm2d_cfie", g.points, g.weights, g.normals, g.curvature, identity=0.5,
                   wavenumber=k, eta=k)


def helm3_prob(g, wavelengths=3.18):
    return Problem("helm3d_sl", g.points, g.weights,
                   wavenumber=W.helmholtz_wavenumber(g, wavelengths))


@pytest.mark.parametrize("mk,leaf", [(lambda: dl_prob(W.star_curve(700)), 32),
                                     (lambda: sl_prob(W.star_curve(500)), 24),
                                     (lambda: sph_prob(W.fibonacci_sphere(600)), 40),
                                     (lambda: helm3_prob(W.fibonacci_sphere(500)), 40)])
def test_eps_zero_is_dense_lu(mk, leaf):
    p = mk()
    F = factor(p, 0.0, leaf, 64 if p.dim == 2 else 128)
    for r in F.records.values():
        assert r.k == r.n
    assert F.root_size == p.n
    b = W.gaussian_rhs(p.n, 3, 5, p.is_complex)
    x = F.solve(b)
    xd = dense.solve(p, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-12


@pytest.mark.parametrize("kind,n,eps,leaf", [("dl", 1024, 1e-9, 64), ("dl", 2048, 1e-6, 32),
                                             ("sl", 1024, 1e-9, 64), ("sl", 1024, 1e-12, 64)])
def test_brute_force_error_bounds(kind, n, eps, leaf):
    g = W.star_curve(n)
    p = dl_prob(g) if kind == "dl" else sl_prob(g)
    npx = 64 if eps >= 1e-9 else 96
    F = factor(p, eps, leaf, npx)
    A = dense.matrix(p)
    kappa = np.linalg.cond(A)
    b = W.gaussian_rhs(n, 2, 1)
    x = F.solve(b)
    xd = np.linalg.solve(A, b)
    rel = np.linalg.norm(x - xd) / np.linalg.norm(xd)
    res = np.linalg.norm(A @ x - b) / np.linalg.norm(b)
    assert rel <= 2 * eps * kappa / (1 - eps * kappa)
    assert res <= eps * kappa
    if kind == "dl":       # second kind: O(eps) outright
        assert rel <= 10 * eps and res <= 10 * eps


@pytest.mark.parametrize("mk,eps,leaf", [(lambda: dl_prob(W.star_curve(1024)), 1e-9, 64),
                                         (lambda: sl_prob(W.star_curve(700)), 1e-6, 32),
                                         (lambda: helm_prob(W.star_curve(800)), 1e-9, 64),
                                         (lambda: sph_prob(W.fibonacci_sphere(900)), 1e-4, 48)])
def test_sparse_embedding_equals_telescoping_inverse(mk, eps, leaf):
    p = mk()
    F = factor(p, eps, leaf, 64 if p.dim == 2 else 128)
    b = W.gaussian_rhs(p.n, 2, 2)
    x = F.solve(b)
    xe = embedding_solve(F, b)
    assert np.linalg.norm(x - xe) / np.linalg.norm(x) < 1e-12
    # the compressed forward operator maps the solution back to b
    assert np.linalg.norm(compressed_matvec(F, x) - b) / np.linalg.norm(b) < 1e-12


def test_compressed_operator_close_to_A():
    g = W.star_curve(1024)
    p = dl_prob(g)
    F = factor(p, 1e-9, 64, 64)
    A = dense.matrix(p)
    rng = np.random.default_rng(0)
    for _ in range(3):
        v = rng.standard_normal(p.n)
        y = compressed_matvec(F, v)
        assert np.linalg.norm(y - A @ v) / np.linalg.norm(A @ v) < 1e-8


@pytest.mark.parametrize("mk", [lambda g: sl_prob(g), lambda g: helm_prob(g)])
def test_lambda_equals_schur_complement(mk):
    g = W.star_curve(1024)
    F = factor(mk(g), 1e-9, 64, 64)
    checked = 0
    for r in F.records.values():
        k, n = r.k, r.n
        if not (0 < k < n):
            continue
        s, rr, T = r.idr.skel, r.idr.redund, r.idr.T
        D = r.D
        Xrr = D[np.ix_(rr, rr)] - T.T @ D[np.ix_(s, rr)] - D[np.ix_(rr, s)] @ T \
            + T.T @ D[np.ix_(s, s)] @ T
        Xrs = D[np.ix_(rr, s)] - T.T @ D[np.ix_(s, s)]
        Xsr = D[np.ix_(s, rr)] - D[np.ix_(s, s)] @ T
        Xss = D[np.ix_(s, s)]
        schur = Xss - Xsr @ np.linalg.solve(Xrr, Xrs)
        assert np.linalg.norm(schur - r.Lam) <= 1e-9 * np.linalg.norm(r.Lam)
        # cD = [I; -T] X_rr^-1 [I, -T^T] in (r, s) coordinates
        G = np.linalg.inv(Xrr)
        Pr = np.zeros((n, rr.size), dtype=D.dtype)
        Pr[rr, np.arange(rr.size)] = 1.0
        Pr[np.ix_(s, np.arange(rr.size))] = -T
        cD = Pr @ G @ Pr.T
        assert np.linalg.norm(cD - r.cD) <= 1e-8 * np.linalg.norm(r.cD)
        checked += 1
    assert checked > 10


def test_proxy_compression_valid_against_true_far_field():
    # One-level check (Section 3.2): the skeletons chosen from near + proxy rows
    # reproduce the true interactions with every far DOF to ~eps.
    g = W.star_curve(2048)
    for p, eps in ((sl_prob(g), 1e-9), (dl_prob(g), 1e-9)):
        F = factor(p, eps, 64, 64)
        t = F.tree
        d = t.maxdepth
        allidx = np.arange(p.n)
        worst = 0.0
        boxes = [b for b in t.boxes_at(d) if 0 < F.records[b].k < F.records[b].n][:12]
        assert len(boxes) >= 6
        for b in boxes:
            r = F.records[b]
            rho = 1.5 * t.side[b]
            near = near_dofs(F.prob.points, allidx, r.J, t.center[b], rho)
            far = np.setdiff1d(allidx, np.concatenate([near, r.J]))
            out = block(F.prob, far, r.J)           # far targets <- box sources
            inc = block(F.prob, r.J, far).T         # box targets <- far sources
            M = compression_block(F.prob, r.J, near, t.center[b], rho, 64)
            scale = np.linalg.norm(M, 2)
            for blk in (out, inc):
                res = blk[:, r.idr.redund] - blk[:, r.idr.skel] @ r.idr.T
                worst = max(worst, np.linalg.norm(res, 2) / scale)
        assert worst < 100 * eps


def test_interior_dirichlet_point_source():
    # Section 6.2: boundary data from an exterior point source; the double-layer
    # solution evaluated inside must match the source's field.
    g = W.ellipse(2048)
    p = dl_prob(g)
    F = factor(p, 1e-9, 64, 64)
    src = np.array([[3.0, 2.0]])
    lap = Problem("lap2d_sl", g.points, g.weights)
    f = kernel(lap, g.points, src)[:, 0]
    sigma = F.solve(f)
    xin = np.array([[0.3, -0.2]])
    u = (kernel(p, xin, g.points, g.normals) * g.weights) @ sigma
    exact = kernel(lap, xin, src)[0, 0]
    assert abs(u[0] - exact) / abs(exact) < 1e-9


def test_sphere_solve_brute_force():
    g = W.fibonacci_sphere(1500)
    p = sph_prob(g)
    F = factor(p, 1e-6, 128, 256)
    A = dense.matrix(p)
    b = W.gaussian_rhs(p.n, 1, 3)
    x = F.solve(b)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1e-6 * kappa
    assert np.linalg.norm(x - np.linalg.solve(A, b)) / np.linalg.norm(x) <= 2e-6 * kappa


def test_helmholtz3d_sphere_brute_force():
    # Section 5's bounds against dense Gaussian elimination for the 3D Helmholtz single
    # layer at the paper's 3D frequency (3.18 wavelengths across the sphere)
    g = W.fibonacci_sphere(1200)
    p = helm3_prob(g)
    F = factor(p, 1e-6, 128, 256)
    A = dense.matrix(p)
    b = W.gaussian_rhs(p.n, 1, 4, True)
    x = F.solve(b)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1e-6 * kappa
    assert np.linalg.norm(x - np.linalg.solve(A, b)) / np.linalg.norm(x) <= 2e-6 * kappa


def test_ranks_consistent_with_paper_scale():
    # Table 5 reports O(30) top-level skeletons for a 2D curve at eps = 1e-9,
    # essentially independent of N; with four depth-1 boxes the root here holds
    # a few tens per box, and it must not grow with N.
    sizes = []
    for n in (1024, 4096):
        F = factor(dl_prob(W.star_curve(n)), 1e-9, 64, 64)
        sizes.append(F.root_size)
    assert all(40 <= s <= 260 for s in sizes)
    assert sizes[1] <= 1.3 * sizes[0]


def test_helmholtz_cfie_brute_force():
    # complex128 path: RS solution of the combined-field system against dense LU, and
    # the second-kind bound (relative error and residual O(eps)).
    g = W.star_curve(1024)
    p = helm_prob(g, 5.0)
    eps = 1e-9
    F = factor(p, eps, 64, 64)
    A = dense.matrix(p)
    b = W.gaussian_rhs(p.n, 2, 3, complex_valued=True)
    x = F.solve(b)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 10 * eps
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 10 * eps
    assert any(0 < r.k < r.n for r in F.records.values())


@pytest.mark.parametrize("mk,eps,leaf,npx", [(lambda: dl_prob(W.star_curve(1500)), 1e-9, 64, 64),
                                            (lambda: sph_prob(W.fibonacci_sphere(1500)), 1e-6, 128, 256)])
def test_sketched_id_factorization_brute_force(mk, eps, leaf, npx):
    # Compression through random row sketches (the paper's randomized ID): the solve
    # still meets Section 5's bounds against dense Gaussian elimination.
    p = mk()
    F = factor(p, eps, leaf, npx, id_mode="sketch", sketch_seed=77)
    A = dense.matrix(p)
    b = W.gaussian_rhs(p.n, 1, 6)
    x = F.solve(b)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 10 * eps * kappa
    assert np.linalg.norm(x - np.linalg.solve(A, b)) / np.linalg.norm(x) <= 20 * eps * kappa
    # a different seed gives a different (equally valid) compression
    F2 = factor(p, eps, leaf, npx, id_mode="sketch", sketch_seed=78)
    assert any(not np.array_equal(F.records[b].skel, F2.records[b].skel) for b in F.records)
