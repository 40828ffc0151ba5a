"""The C ABI's contract on the MI355X: pointer kinds, stream order, busy handles and the
singular-pivot report.

* rs_solve on host memory is synchronous and gives bitwise the device result;
* the server accepts device memory only, and a request runs after the work its
  producer had queued on its stream when it submitted;
* rs_free refuses (RS_EBUSY) a handle whose solve is still queued on a stream;
* an exactly singular system is reported as RS_ESINGULAR naming the tree depth and
  box of the failing elimination.  The systems are singular by construction: on a
  straight segment with normals perpendicular to it the double-layer kernel
  (x - y).nu_y / (2 pi |x - y|^2) is exactly zero, and with zero curvature and no
  identity term so is every diagonal entry, so A = 0 in floating point.
"""
import ctypes as C
import re

import numpy as np
import pytest

import workloads as W
from parity_util import to_device

pytestmark = pytest.mark.gpu


def _star_dl(rs, n, eps=1e-9, leaf=64):
    g = W.star_curve(n)
    t = rs.build_tree(g.points, leaf)
    h = rs.factor("lap2d_dl", t, g.points, g.weights, eps, normals=g.normals,
                  curvature=g.curvature, identity=-0.5, proxy_points=64)
    return g, h


def _busy_work(torch, stream, n=3072, reps=6):
    """FP64 products queued on `stream` (a few tens of milliseconds of device work)."""
    with torch.cuda.stream(stream):
        X = torch.rand(n, n, dtype=torch.float64, device="cuda") / n
        Y = torch.empty_like(X)
        for _ in range(reps):
            torch.mm(X, X, out=Y)
            torch.mm(Y, X, out=X)
    return X


def test_host_pointer_solve_matches_device(gpu_lib):
    import torch
    rs = gpu_lib
    g, h = _star_dl(rs, 3000)
    b = W.gaussian_rhs(g.n, 7, 3)
    B = to_device(b)
    h.solve(B)
    torch.cuda.synchronize()
    xd = B.cpu().numpy()
    xh = h.solve_host(b)
    assert np.array_equal(xh, xd)
    # leading dimension larger than n, one column
    xv = h.solve_host(b[:, 2])
    assert np.array_equal(xv, xd[:, 2])


def test_free_refused_while_solve_queued(gpu_lib):
    import torch
    rs = gpu_lib
    g, h = _star_dl(rs, 4096)
    s = torch.cuda.Stream()
    B = to_device(W.gaussian_rhs(g.n, 4, 9))
    torch.cuda.synchronize()
    keep = _busy_work(torch, s)
    h.solve(B, stream=s)
    with pytest.raises(rs.RSError) as e:
        h.free()
    assert e.value.code == rs.RS_EBUSY
    s.synchronize()
    h.free()
    del keep


def test_server_rejects_host_memory(gpu_lib):
    import torch
    rs = gpu_lib
    g, h = _star_dl(rs, 2000)
    srv = rs.Server(1 << 30)
    with pytest.raises(TypeError):
        srv.submit_solve(h, torch.zeros(g.n, 1, dtype=torch.float64))
    host = np.zeros(g.n)
    t = C.c_uint64()
    st = rs.binding._lib.rs_server_submit_solve(srv._s, h.handle, C.c_void_p(host.ctypes.data),
                                                g.n, 1, None, C.byref(t))
    assert st == rs.RS_EINVAL
    srv.close()


def test_server_waits_for_producer_stream(gpu_lib):
    import torch
    rs = gpu_lib
    g, h = _star_dl(rs, 4096)
    b = W.gaussian_rhs(g.n, 16, 21)
    ref = to_device(b)
    h.solve(ref)
    src = to_device(b)
    torch.cuda.synchronize()
    srv = rs.Server(1 << 30)
    s = torch.cuda.Stream()
    B = torch.zeros(16, g.n, dtype=torch.float64, device="cuda").t()
    keep = _busy_work(torch, s)
    with torch.cuda.stream(s):
        B.copy_(src)                  # written on s after tens of ms of other work
    tk = srv.submit_solve(h, B, stream=s)
    srv.wait(tk)
    torch.cuda.synchronize()
    assert torch.equal(B, ref)
    srv.close()
    del keep


def _collinear(n):
    x = (np.arange(n, dtype=np.float64) + 0.5) / n
    pts = np.stack([x, np.zeros(n)], axis=1)
    nrm = np.tile(np.array([0.0, 1.0]), (n, 1))
    return pts, nrm, np.zeros(n), np.full(n, 1.0 / n)


@pytest.mark.parametrize("eps", [1e-9, 0.0])
def test_singular_pivot_names_depth_and_box(gpu_lib, eps):
    rs = gpu_lib
    n, leaf = 600, 32
    pts, nrm, kap, w = _collinear(n)
    t = rs.build_tree(pts, leaf)
    with pytest.raises(rs.RSError) as e:
        rs.factor("lap2d_dl", t, pts, w, eps, normals=nrm, curvature=kap, identity=0.0,
                  proxy_points=64)
    assert e.value.code == rs.RS_ESINGULAR
    m = re.search(r"depth (\d+), box (\d+)", str(e.value))
    assert m, str(e.value)
    depth, box = int(m.group(1)), int(m.group(2))
    tr = t.export()
    assert 0 <= box < tr["depth"].size and tr["depth"][box] == depth
    if eps == 0.0:
        # no compression: every unknown reaches the root, which is the zero matrix
        assert (depth, box) == (0, 0) and "root" in str(e.value)
    else:
        # every diagonal block is zero: the failing box is one that was compressed
        assert depth >= 1
