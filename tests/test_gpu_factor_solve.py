"""Factor and solve in one call (rs_factor_solve_ex) on the MI355X.

The solve's permutation and each level's upward sweep run on another stream as soon
as that level is factored, and the root block is inverted beside them; the results must
be those of rs_factor_ex followed by rs_solve_ex bit for bit (the same kernels on the
same data): solutions, ranks and the handle's later solves, in both launch modes, for
real and complex operators, with boxes in every sweep class.  A singular system is
reported as by rs_factor_ex (the root named).
"""
import re

import numpy as np
import pytest

import workloads as W
from parity_util import to_device

pytestmark = pytest.mark.gpu


def _two_ways(rs, dtype, kind, t, g, eps, b, mode, **kw):
    import torch
    h = rs.factor(kind, t, g.points, g.weights, eps, launch_mode=mode, **kw)
    B1 = to_device(b, dtype)
    h.solve(B1, launch_mode=mode)
    B2 = to_device(b, dtype)
    h2 = rs.factor_solve(kind, t, g.points, g.weights, eps, B2, launch_mode=mode, **kw)
    torch.cuda.synchronize()
    return h, h2, B1.cpu().numpy(), B2.cpu().numpy()


@pytest.mark.parametrize("mode", ["level", "per_box"])
def test_factor_solve_real_bitwise(gpu_lib, mode):
    import torch
    rs = gpu_lib
    n = 8192 if mode == "level" else 2048
    g = W.star_curve(n)
    t = rs.build_tree(g.points, 64)
    for nrhs in (1, 64, 130):
        b = W.gaussian_rhs(n, nrhs, 300 + nrhs)
        h, h2, x1, x2 = _two_ways(rs, None, "lap2d_sl", t, g, 1e-9, b, mode, proxy_points=64)
        assert np.array_equal(x1, x2), nrhs
        assert h.stats()["root_size"] == h2.stats()["root_size"]
        assert h.stats()["total_skeletons"] == h2.stats()["total_skeletons"]
        # the handle of the combined call solves like the other one
        c = W.gaussian_rhs(n, 3, 7)
        C1, C2 = to_device(c), to_device(c)
        h.solve(C1)
        h2.solve(C2)
        torch.cuda.synchronize()
        assert torch.equal(C1, C2)
        h.free()
        h2.free()


def test_factor_solve_sphere_and_complex_bitwise(gpu_lib):
    import torch
    rs = gpu_lib
    gs = W.fibonacci_sphere(4000)
    ts = rs.build_tree(gs.points, 128)
    b = W.gaussian_rhs(4000, 5, 11)
    _, _, x1, x2 = _two_ways(rs, None, "lap3d_sl", ts, gs, 1e-6, b, "level", proxy_points=256)
    assert np.array_equal(x1, x2)
    g = W.star_curve(4000)
    t = rs.build_tree(g.points, 64)
    k = W.helmholtz_wavenumber(g, 4.0)
    b = W.gaussian_rhs(4000, 9, 13, complex_valued=True)
    _, _, x1, x2 = _two_ways(rs, torch.complex128, "helm2d_cfie", t, g, 1e-9, b, "level",
                             normals=g.normals, curvature=g.curvature, identity=0.5,
                             wavenumber=k, eta=k, proxy_points=64)
    assert np.array_equal(x1, x2)


@pytest.mark.parametrize("kind,n,leaf", [("lap2d_sl", 6000, 900), ("helm2d_cfie", 4000, 330)])
def test_factor_solve_wide_boxes_bitwise(gpu_lib, kind, n, leaf):
    # leaves above the MFMA sweep class: the upward sweeps that run beside the
    # factorization stage those boxes through the wide path's scratch
    import torch
    rs = gpu_lib
    g = W.star_curve(n)
    t = rs.build_tree(g.points, leaf)
    cplx = kind == "helm2d_cfie"
    kw = dict(proxy_points=64)
    if cplx:
        k = W.helmholtz_wavenumber(g, 6.0)
        kw.update(normals=g.normals, curvature=g.curvature, identity=0.5, wavenumber=k, eta=k)
    for nrhs in (1, 17, 100):
        b = W.gaussian_rhs(n, nrhs, 90 + nrhs, complex_valued=cplx)
        h, h2, x1, x2 = _two_ways(rs, torch.complex128 if cplx else None, kind, t, g, 1e-9, b,
                                  "level", **kw)
        assert np.array_equal(x1, x2), nrhs
        h.free()
        h2.free()


def test_factor_solve_singular_and_arguments(gpu_lib):
    import torch
    rs = gpu_lib
    n = 600
    x = (np.arange(n, dtype=np.float64) + 0.5) / n
    pts = np.stack([x, np.zeros(n)], axis=1)
    nrm = np.tile(np.array([0.0, 1.0]), (n, 1))
    t = rs.build_tree(pts, 32)
    B = torch.zeros(n, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(rs.RSError) as e:
        rs.factor_solve("lap2d_dl", t, pts, np.full(n, 1.0 / n), 0.0, B, normals=nrm,
                        curvature=np.zeros(n), identity=0.0, proxy_points=64)
    assert e.value.code == rs.RS_ESINGULAR
    assert re.search(r"depth 0, box 0", str(e.value)) and "root" in str(e.value)
    g = W.star_curve(512)
    t2 = rs.build_tree(g.points, 32)
    with pytest.raises(TypeError):
        rs.factor_solve("lap2d_sl", t2, g.points, g.weights, 1e-9,
                        torch.zeros(512, 2, dtype=torch.float64))          # host tensor
    with pytest.raises(ValueError):
        rs.factor_solve("lap2d_sl", t2, g.points, g.weights, 1e-9,
                        torch.zeros(511, 2, dtype=torch.float64, device="cuda"))
