"""3D Helmholtz single layer (Section 6.1 eq. (3d-helmholtz), complex128) on the MI355X.

The sphere workload of the paper's 3D Helmholtz experiments: Fibonacci points on the unit
sphere, G_k = exp(i k r) / (4 pi r), 3.18 wavelengths across the sphere (the frequency of
the paper's 3D solver runs), eps = 1e-6, octree leaf 128.  The same kernels as the
Laplace path run on complex128 entries; boxes above the small classes take the
multi-workgroup ID and, at N = 2048 with 256 proxies, a root of more than 1536 unknowns
(the root inversion spread over launches).  Criteria as for the other kernels: skeleton
sets equal wherever no tie can reach a box, solutions within 10 eps of the oracle's when
all skeletons agree, residual below 10 eps (the discretized operator has condition number
about 13 at this frequency), bitwise equality in batches with other complex problems.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Problem, dense
from oracle import factor as ofactor
from parity_util import compare_skeletons, identical_skeletons, to_device

pytestmark = pytest.mark.gpu


def _setup(rs, n, eps, npx=256, wavelengths=3.18, leaf=128):
    g = W.fibonacci_sphere(n)
    k = W.helmholtz_wavenumber(g, wavelengths)
    p = Problem("helm3d_sl", g.points, g.weights, wavenumber=k)
    t = rs.build_tree(g.points, leaf)
    h = rs.factor("helm3d_sl", t, g.points, g.weights, eps, proxy_points=npx, wavenumber=k)
    return g, k, p, t, h


def _solve(h, b):
    import torch
    B = to_device(b, torch.complex128)
    h.solve(B)
    torch.cuda.synchronize()
    return B.cpu().numpy()


def test_helmholtz3d_parity(gpu_lib):
    rs = gpu_lib
    eps = 1e-6
    g, k, p, t, h = _setup(rs, 2048, eps)
    assert h.is_complex and h.stats()["dim"] == 3
    F = ofactor(p, eps, 128, 256)
    compared, tied = compare_skeletons(h, F)
    same = identical_skeletons(h, F)
    assert compared >= 0.9 * len(F.records)
    if same:
        assert h.stats()["root_size"] == F.root_size
    b = W.gaussian_rhs(g.n, 3, 8, complex_valued=True)
    x = _solve(h, b)
    xo = F.solve(b)
    if same:
        assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 10 * eps
    A = dense.matrix(p)
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 10 * eps


def test_helmholtz3d_eps_zero_is_dense_lu(gpu_lib):
    rs = gpu_lib
    g, k, p, t, h = _setup(rs, 600, 0.0, leaf=64)
    assert h.stats()["root_size"] == 600
    b = W.gaussian_rhs(600, 4, 9, complex_valued=True)
    x = _solve(h, b)
    xd = dense.solve(p, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-11


def test_helmholtz3d_batched_with_2d_complex_bitwise(gpu_lib):
    import torch
    rs = gpu_lib
    g3 = W.fibonacci_sphere(1500)
    k3 = W.helmholtz_wavenumber(g3, 2.0)
    g2 = W.star_curve(2500)
    k2 = W.helmholtz_wavenumber(g2, 5.0)
    t3, t2 = rs.build_tree(g3.points, 128), rs.build_tree(g2.points, 64)
    probs = [dict(kind="helm3d_sl", tree=t3, points=g3.points, weights=g3.weights, eps=1e-6,
                  proxy_points=256, wavenumber=k3),
             dict(kind="helm2d_cfie", tree=t2, points=g2.points, weights=g2.weights, eps=1e-9,
                  normals=g2.normals, curvature=g2.curvature, identity=0.5, wavenumber=k2,
                  eta=k2)]
    hb = rs.factor_batched(probs)
    h3 = rs.factor("helm3d_sl", t3, g3.points, g3.weights, 1e-6, proxy_points=256,
                   wavenumber=k3)
    k_b, s_b = hb[0].box_skeletons()
    k_s, s_s = h3.box_skeletons()
    assert np.array_equal(k_b, k_s)
    b = W.gaussian_rhs(g3.n, 5, 12, complex_valued=True)
    assert np.array_equal(_solve(hb[0], b), _solve(h3, b))
    b2 = W.gaussian_rhs(g2.n, 2, 13, complex_valued=True)
    B1, B2 = to_device(b, torch.complex128), to_device(b2, torch.complex128)
    rs.solve_batched(hb, [B1, B2])
    torch.cuda.synchronize()
    assert np.array_equal(B1.cpu().numpy(), _solve(h3, b))


def test_single_scatterer_factors_as_block_preconditioner(gpu_lib):
    """The multiple-scattering example's preconditioner (Section 6.4): two copies of the
    scatterer r = (2 + cos 3t)/6, ten wavelengths in size, each factored on its own
    (exterior combined field, eps = 1e-6); P^{-1} = diag(A_11^{-1}, A_22^{-1}) applied by
    one batched solve over the two handles inverts the block-diagonal part of the coupled
    system: P^{-1} (diag(A_11, A_22) x) = x to the compression precision, and each block
    equals its single solve bitwise."""
    import torch
    rs = gpu_lib
    n, eps = 1024, 1e-6
    gs = [W.scatterer_curve(n, (-0.6, 0.0)), W.scatterer_curve(n, (0.6, 0.0))]
    k = W.helmholtz_wavenumber(gs[0], 10.0)
    hs, ps = [], []
    for g in gs:
        t = rs.build_tree(g.points, 64)
        # proxy circles of the top boxes are ~47 radians around: 160 points resolve them
        hs.append(rs.factor("helm2d_cfie", t, g.points, g.weights, eps, normals=g.normals,
                            curvature=g.curvature, identity=0.5, wavenumber=k, eta=k,
                            proxy_points=160))
        ps.append(Problem("helm2d_cfie", g.points, g.weights, g.normals, g.curvature,
                          identity=0.5, wavenumber=k, eta=k))
    xs = [W.gaussian_rhs(n, 2, 30 + i, complex_valued=True) for i in range(2)]
    As = [dense.matrix(p) for p in ps]
    bs = [A @ x for A, x in zip(As, xs)]
    Bs = [to_device(b, torch.complex128) for b in bs]
    rs.solve_batched(hs, Bs)
    torch.cuda.synchronize()
    for i in range(2):
        y = Bs[i].cpu().numpy()
        kappa = np.linalg.cond(As[i])
        assert np.linalg.norm(y - xs[i]) / np.linalg.norm(xs[i]) <= 10 * eps * kappa
        assert np.array_equal(y, _solve(hs[i], bs[i]))
