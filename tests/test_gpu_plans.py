"""Graph-captured solve plans and the sweep tile-width autotuner (MI355X).

A plan replays the per-level sweep launches captured once into a HIP graph; every
replay must equal rs_solve bitwise, also with the program's own eager work and
synchronizations between replays.  The autotuner changes tile widths only, so solves
before and after tuning are bitwise identical; a saved table loads back unchanged.
"""
import numpy as np
import pytest

import workloads as W
from parity_util import to_device

pytestmark = pytest.mark.gpu


def _laplace(rs, n, kind="lap2d_sl"):
    g = W.star_curve(n) if kind == "lap2d_sl" else W.random_curve(n, [0.03, 0.02], [0.4, 1.1])
    t = rs.build_tree(g.points, 64)
    kw = {}
    if kind == "lap2d_dl":
        kw = dict(normals=g.normals, curvature=g.curvature, identity=-0.5)
    return rs.factor(kind, t, g.points, g.weights, 1e-9, **kw), t


def _eager(h, b, dtype):
    import torch
    B = to_device(b, dtype)
    h.solve(B)
    torch.cuda.synchronize()
    return B.cpu().numpy()


def test_plan_replays_equal_eager_solves(gpu_lib):
    import torch
    rs = gpu_lib
    h1, _ = _laplace(rs, 8192)
    h2, _ = _laplace(rs, 3000, "lap2d_dl")
    g3 = W.star_curve(2048)
    k3 = W.helmholtz_wavenumber(g3, 6.0)
    t3 = rs.build_tree(g3.points, 64)
    h3 = rs.factor("helm2d_cfie", t3, g3.points, g3.weights, 1e-9, normals=g3.normals,
                   curvature=g3.curvature, identity=0.5, wavenumber=k3, eta=k3)
    B1 = to_device(np.zeros((8192, 1)), torch.float64)
    B2 = to_device(np.zeros((3000, 37)), torch.float64)
    B3 = to_device(np.zeros((2048, 5), dtype=np.complex128), torch.complex128)
    plan = rs.Plan([h1, h2, h3], [B1, B2, B3])
    for rep in range(4):
        b1 = W.gaussian_rhs(8192, 1, 100 + rep)
        b2 = W.gaussian_rhs(3000, 37, 200 + rep)
        b3 = W.gaussian_rhs(2048, 5, 300 + rep, complex_valued=True)
        B1.copy_(to_device(b1, torch.float64))
        B2.copy_(to_device(b2, torch.float64))
        B3.copy_(to_device(b3, torch.complex128))
        plan.launch()
        torch.cuda.synchronize()
        assert np.array_equal(B1.cpu().numpy(), _eager(h1, b1, torch.float64))
        assert np.array_equal(B2.cpu().numpy(), _eager(h2, b2, torch.float64))
        assert np.array_equal(B3.cpu().numpy(), _eager(h3, b3, torch.complex128))
        _ = (torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")).sum()
    # the handles are busy while the plan exists
    with pytest.raises(rs.RSError):
        h1.free()
    plan.free()
    h1.free()


def test_plan_argument_errors(gpu_lib):
    import torch
    rs = gpu_lib
    h, _ = _laplace(rs, 1024)
    with pytest.raises(ValueError):
        rs.Plan([h], [torch.zeros(1023, 1, dtype=torch.float64, device="cuda")])
    with pytest.raises(TypeError):
        rs.Plan([h], [torch.zeros(1024, 1, dtype=torch.complex128, device="cuda")])


def test_autotune_changes_speed_not_results(gpu_lib, tmp_path):
    import torch
    rs = gpu_lib
    rs.tune_clear()
    h, _ = _laplace(rs, 16384)
    b = W.gaussian_rhs(16384, 48, 5)
    before = _eager(h, b, torch.float64)
    rs.autotune(h, (1, 48, 200), reps=2)
    table = rs.tune_entries()
    assert table and all(w in (1, 4, 16, 32, 64) for w in table.values())
    after = _eager(h, b, torch.float64)
    assert np.array_equal(before, after)
    path = str(tmp_path / "tune.txt")
    rs.tune_save(path)
    rs.tune_clear()
    assert rs.tune_entries() == {}
    rs.tune_load(path)
    assert rs.tune_entries() == table
    bad = tmp_path / "bad.txt"
    bad.write_text("1 7\n")
    with pytest.raises(rs.RSError):
        rs.tune_load(str(bad))
    rs.tune_clear()
