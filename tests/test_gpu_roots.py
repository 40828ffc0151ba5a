"""Roots and box inversions at the edges of the register Gauss-Jordan classes, on the MI355X.

eps = 0 keeps every unknown, so the whole system is the root and the solve is dense
Gaussian elimination's (the root block of Section 3.4, eq. (multilevel-inverse)).  Real
roots of up to 64 unknowns are inverted in registers inside the box factorization, real
roots of 65 to 200 unknowns by their own register kernel, larger ones by the blocked
elimination; a complex root in the same range takes the blocked elimination.  Criteria:
the dense solution within 1e-11 (real) or 1e-10 (complex), and the same bits from a
per-box launch, a batched factorization and a second factorization.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Problem, dense
from parity_util import to_device

pytestmark = pytest.mark.gpu


def _solve(h, b, dtype=None, mode="level"):
    import torch
    B = to_device(b, dtype)
    h.solve(B, launch_mode=mode)
    torch.cuda.synchronize()
    return B.cpu().numpy()


@pytest.mark.parametrize("n", [40, 64, 65, 150, 200, 201])
def test_real_root_classes_eps_zero(gpu_lib, n):
    rs = gpu_lib
    g = W.star_curve(n)
    p = Problem("lap2d_sl", g.points, g.weights)
    t = rs.build_tree(g.points, 16)
    h = rs.factor("lap2d_sl", t, g.points, g.weights, 0.0, proxy_points=64)
    assert h.stats()["root_size"] == n
    h2 = rs.factor("lap2d_sl", t, g.points, g.weights, 0.0, proxy_points=64,
                   launch_mode="per_box")
    hb = rs.factor_batched([dict(kind="lap2d_sl", tree=t, points=g.points, weights=g.weights,
                                 eps=0.0, proxy_points=64)] * 2)
    for nrhs in (1, 7):
        b = W.gaussian_rhs(n, nrhs, 90 + n + nrhs)
        x = _solve(h, b)
        xd = dense.solve(p, b)
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-11, (n, nrhs)
        assert np.array_equal(x, _solve(h2, b, mode="per_box"))
        for hh in hb:
            assert np.array_equal(x, _solve(hh, b))


@pytest.mark.parametrize("n", [100, 180])
def test_complex_root_mid_size_eps_zero(gpu_lib, n):
    import torch
    rs = gpu_lib
    g = W.star_curve(n)
    k = W.helmholtz_wavenumber(g, 2.0)
    p = Problem("helm2d_cfie", g.points, g.weights, g.normals, g.curvature, identity=0.5,
                wavenumber=k, eta=k)
    t = rs.build_tree(g.points, 16)
    h = rs.factor("helm2d_cfie", t, g.points, g.weights, 0.0, normals=g.normals,
                  curvature=g.curvature, identity=0.5, wavenumber=k, eta=k)
    assert h.stats()["root_size"] == n
    b = W.gaussian_rhs(n, 3, 7 + n, complex_valued=True)
    x = _solve(h, b, torch.complex128)
    xd = dense.solve(p, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10
