"""rs_solve_noalloc: the solve with its workspace in the library's fixed per-device
scratch array (no device allocation) equals rs_solve bitwise.

Two calls in a row share the scratch; the second is smaller than the first, so it
runs over what the first left behind.  A case with a box above the small-box sweep
class (eps = 0 puts every unknown at the root) exercises the wide-box staging that
follows the workspace in the scratch.  A request over the scratch's size is refused.
"""
import numpy as np
import pytest

import workloads as W
from parity_util import to_device

pytestmark = pytest.mark.gpu


def _factor(rs, kind, n, eps, leaf=64):
    g = W.star_curve(n)
    t = rs.build_tree(g.points, leaf)
    kw = {}
    if kind == "lap2d_dl":
        kw = dict(normals=g.normals, curvature=g.curvature, identity=-0.5)
    return g, rs.factor(kind, t, g.points, g.weights, eps, proxy_points=64, **kw)


def _both(h, b):
    import torch
    B1 = to_device(b)
    B2 = to_device(b)
    h.solve(B1)
    h.solve_noalloc(B2)
    torch.cuda.synchronize()
    return B1.cpu().numpy(), B2.cpu().numpy()


def test_noalloc_equals_solve_two_calls(gpu_lib):
    rs = gpu_lib
    g1, h1 = _factor(rs, "lap2d_dl", 4096, 1e-9)
    g2, h2 = _factor(rs, "lap2d_sl", 2500, 1e-9, leaf=48)
    x1, y1 = _both(h1, W.gaussian_rhs(g1.n, 64, 31))
    assert np.array_equal(x1, y1)
    x2, y2 = _both(h2, W.gaussian_rhs(g2.n, 3, 32))
    assert np.array_equal(x2, y2)


def test_noalloc_wide_root(gpu_lib):
    rs = gpu_lib
    g, h = _factor(rs, "lap2d_sl", 700, 0.0, leaf=32)
    assert h.stats()["root_size"] == 700          # above the small-box sweep class
    x, y = _both(h, W.gaussian_rhs(g.n, 40, 33))
    assert np.array_equal(x, y)
    x, y = _both(h, W.gaussian_rhs(g.n, 2, 34))
    assert np.array_equal(x, y)


def test_noalloc_over_limit_refused(gpu_lib):
    import torch
    rs = gpu_lib
    g, h = _factor(rs, "lap2d_dl", 16384, 1e-9)
    B = torch.zeros(1024, g.n, dtype=torch.float64, device="cuda").t()   # 128 MiB
    with pytest.raises(rs.RSError) as e:
        h.solve_noalloc(B)
    assert e.value.code == rs.RS_EINVAL and "scratch" in str(e.value)
