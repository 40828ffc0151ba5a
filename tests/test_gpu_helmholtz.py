"""Helmholtz combined-field (complex128) path on the MI355X against the oracle.

The exterior combined-field system (1/2 I + D_k - i eta S_k) sigma = f on the star curve
(Section 6.1 eq. (2d-helmholtz), the combined layer of Section 3.2) goes through the same
kernels as the Laplace path with complex128 entries.  Parity criteria are those of the
Laplace cases: skeletons equal where the oracle has no tie, T within the conditioning
of R11, solutions within 10 eps of the oracle's, residuals below 10 eps.  The serving
size (N = 32768, 10 wavelengths across) is compared with a stored oracle run in
tests/test_gpu_fullsize.py.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Problem, dense
from oracle import factor as ofactor
from parity_util import compare_skeletons, identical_skeletons, to_device

pytestmark = pytest.mark.gpu


def _oracle_problem(g, k):
    return Problem("helm2d_cfie", g.points, g.weights, g.normals, g.curvature, identity=0.5,
                   wavenumber=k, eta=k)


def _gpu_factor(rs, g, k, eps, leaf=64, npx=64, mode="level"):
    t = rs.build_tree(g.points, leaf)
    h = rs.factor("helm2d_cfie", t, g.points, g.weights, eps, normals=g.normals,
                  curvature=g.curvature, identity=0.5, proxy_points=npx, launch_mode=mode,
                  wavenumber=k, eta=k)
    return t, h


def _gpu_solve(h, b, mode="level"):
    import torch
    B = to_device(b, torch.complex128)
    h.solve(B, launch_mode=mode)
    torch.cuda.synchronize()
    return B.cpu().numpy()


@pytest.mark.parametrize("n,wavelengths,leaf", [(2048, 10.0, 64), (3000, 5.0, 48)])
def test_helmholtz_parity(gpu_lib, n, wavelengths, leaf):
    rs = gpu_lib
    eps = 1e-9
    g = W.star_curve(n)
    k = W.helmholtz_wavenumber(g, wavelengths)
    p = _oracle_problem(g, k)
    F = ofactor(p, eps, leaf, 64)
    _, h = _gpu_factor(rs, g, k, eps, leaf)
    assert h.is_complex
    compared, tied = compare_skeletons(h, F)
    same = identical_skeletons(h, F)
    assert compared >= 0.9 * len(F.records)
    b = W.gaussian_rhs(n, 3, 7, complex_valued=True)
    x = _gpu_solve(h, b)
    xo = F.solve(b)
    rel = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    if same:
        assert rel <= 10 * eps, rel
    A = dense.matrix(p)
    res = np.linalg.norm(A @ x - b) / np.linalg.norm(b)
    assert res <= 10 * eps, res


def test_helmholtz_multi_rhs_and_launch_modes_bitwise(gpu_lib):
    rs = gpu_lib
    g = W.star_curve(2500)
    k = W.helmholtz_wavenumber(g, 8.0)
    _, h1 = _gpu_factor(rs, g, k, 1e-9, 48, mode="level")
    _, h2 = _gpu_factor(rs, g, k, 1e-9, 48, mode="per_box")
    k1, _ = h1.box_skeletons()
    k2, _ = h2.box_skeletons()
    assert np.array_equal(k1, k2)
    F = ofactor(_oracle_problem(g, k), 1e-9, 48, 64)
    for nrhs in (1, 17, 64, 100):
        b = W.gaussian_rhs(2500, nrhs, 30 + nrhs, complex_valued=True)
        xa = _gpu_solve(h1, b, "level")
        xb = _gpu_solve(h2, b, "per_box")
        assert np.array_equal(xa, xb)
        xo = F.solve(b)
        assert np.linalg.norm(xa - xo) / np.linalg.norm(xo) <= 1e-8


def test_helmholtz_real_rhs_and_dtype_checks(gpu_lib):
    import torch
    rs = gpu_lib
    g = W.star_curve(1024)
    k = W.helmholtz_wavenumber(g, 4.0)
    _, h = _gpu_factor(rs, g, k, 1e-9)
    with pytest.raises(TypeError):
        h.solve(torch.zeros(1024, dtype=torch.float64, device="cuda"))
    b = W.gaussian_rhs(1024, 1, 2)                  # real data, complex solution
    x = _gpu_solve(h, b.astype(np.complex128))
    A = dense.matrix(_oracle_problem(g, k))
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1e-8


def test_mixed_real_and_complex_batches_bitwise(gpu_lib):
    import torch
    rs = gpu_lib
    gh = W.star_curve(3000)
    kh = W.helmholtz_wavenumber(gh, 6.0)
    gl = W.random_curve(2600, [0.03, 0.02], [0.5, 1.5])
    th = rs.build_tree(gh.points, 64)
    tl = rs.build_tree(gl.points, 64)
    probs = [dict(kind="helm2d_cfie", tree=th, points=gh.points, weights=gh.weights, eps=1e-9,
                  normals=gh.normals, curvature=gh.curvature, identity=0.5, wavenumber=kh,
                  eta=kh),
             dict(kind="lap2d_dl", tree=tl, points=gl.points, weights=gl.weights, eps=1e-9,
                  normals=gl.normals, curvature=gl.curvature, identity=-0.5)]
    hb = rs.factor_batched(probs)
    assert hb[0].is_complex and not hb[1].is_complex
    _, hs = _gpu_factor(rs, gh, kh, 1e-9)
    hl = rs.factor("lap2d_dl", tl, gl.points, gl.weights, 1e-9, normals=gl.normals,
                   curvature=gl.curvature, identity=-0.5)
    bh = W.gaussian_rhs(3000, 5, 1, complex_valued=True)
    bl = W.gaussian_rhs(2600, 3, 2)
    Bh = to_device(bh, torch.complex128)
    Bl = to_device(bl, torch.float64)
    rs.solve_batched(hb, [Bh, Bl])
    torch.cuda.synchronize()
    assert np.array_equal(Bh.cpu().numpy(), _gpu_solve(hs, bh))
    Bl2 = to_device(bl, torch.float64)
    hl.solve(Bl2)
    torch.cuda.synchronize()
    assert np.array_equal(Bl.cpu().numpy(), Bl2.cpu().numpy())


def test_server_complex_factor_and_solves(gpu_lib):
    import torch
    rs = gpu_lib
    g = W.star_curve(4096)
    k = W.helmholtz_wavenumber(g, 10.0)
    srv = rs.Server(4 << 30, max_batch_requests=8)
    t = rs.build_tree(g.points, 64)
    tk = srv.submit_factor("helm2d_cfie", t, g.points, g.weights, 1e-9, normals=g.normals,
                           curvature=g.curvature, identity=0.5, wavenumber=k, eta=k)
    hs = srv.wait(tk)
    assert hs.is_complex
    _, hd = _gpu_factor(rs, g, k, 1e-9)
    gl = W.star_curve(2048)
    tl = rs.build_tree(gl.points, 64)
    hl = rs.factor("lap2d_sl", tl, gl.points, gl.weights, 1e-9)
    reqs = []
    for i in range(12):
        if i % 3 == 2:
            b = W.gaussian_rhs(2048, 1 + i, 50 + i)
            reqs.append((hl, b, to_device(b, torch.float64)))
        else:
            b = W.gaussian_rhs(4096, 1 + i, 50 + i, complex_valued=True)
            reqs.append((hs, b, to_device(b, torch.complex128)))
    torch.cuda.synchronize()
    tickets = [srv.submit_solve(h, B) for h, _, B in reqs]
    for tkt in tickets:
        srv.wait(tkt)
    for h, b, B in reqs:
        if h is hs:
            ref = _gpu_solve(hd, b)
        else:
            R = to_device(b, torch.float64)
            hl.solve(R)
            torch.cuda.synchronize()
            ref = R.cpu().numpy()
        assert np.array_equal(B.cpu().numpy(), ref)
    hs.free()
    srv.close()


@pytest.mark.parametrize("n", [130, 300])
def test_helmholtz_eps_zero_is_dense_lu(gpu_lib, n):
    # eps = 0 keeps every DOF: the root is the whole system (blocked Gauss-Jordan
    # inversion), so the solution is dense Gaussian elimination's.
    rs = gpu_lib
    g = W.star_curve(n)
    k = W.helmholtz_wavenumber(g, 3.0)
    _, h = _gpu_factor(rs, g, k, 0.0, 32)
    assert h.stats()["root_size"] == n
    b = W.gaussian_rhs(n, 2, 9, complex_valued=True)
    x = _gpu_solve(h, b)
    xd = dense.solve(_oracle_problem(g, k), b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-11
