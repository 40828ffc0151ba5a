"""Parity with the oracle at the full sizes of the benchmark configurations (MI355X).

* Unit sphere, N = 20480 Fibonacci points, 3D Laplace single layer, eps = 1e-6, octree
  leaf 128, 512 proxies, 64 right-hand sides: against a stored oracle run
  (tests/golden/sphere20480.npz, written by tests/golden/make_fixtures.py, which calls
  only the oracle and the input generators; the oracle needs ~15 min for it).
* Star curve, N = 32768, exterior Helmholtz combined field with 10 wavelengths across,
  eps = 1e-9: against tests/golden/helmholtz32768.npz.
* Star curve, N = 65536, 2D Laplace single layer at eps = 1e-6 (64 proxies) and
  eps = 1e-12 (96 proxies), 512 right-hand sides: against an oracle run in the test.

Criteria (the acceptance tolerance is 10 eps):
* skeleton sets and ranks identical on every box that no tie can reach: no tie at the
  box under the oracle's rule (pivot norms, or the rank decision, closer than 1e-10
  relative plus the rounding width 2 m u |R_00| of Householder QR), none below it, and
  none deciding whether one of its active or near DOFs survives to its depth;
* when every box has the oracle's skeletons (both sides then compress to the same
  A_eps), the device's solution agrees with the oracle's to 10 eps relative per
  compared column;
* residual on sampled rows against the exact matrix: below 10 eps relative to the
  right-hand side for the second-kind Helmholtz system; for the first-kind single
  layers, the device and oracle solutions agree in residual space,
  |A (x - x_oracle)| <= 10 eps |A x_oracle| on the sampled rows, and the device's own
  sampled residual is within 10 eps of |b| wherever the oracle's is.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import Problem, dense
from oracle import factor as ofactor
from parity_util import compare_skeletons, identical_skeletons, to_device, uncertain_boxes

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    path = os.path.join(GOLDEN, name + ".npz")
    assert os.path.exists(path), f"missing fixture {path} (tests/golden/make_fixtures.py)"
    return np.load(path, allow_pickle=False)


def _compare_with_fixture(h, t, g, fx):
    """Per-box ranks and skeleton sets against the stored oracle run, on every box that
    no tie can reach (parity_util.uncertain_boxes; near fields by the oracle's rule,
    |x - c|^2 < (1.5 side)^2); returns (#compared, identical everywhere)."""
    tr = t.export()
    nbox = tr["depth"].size
    assert nbox == int(fx["nbox"]) and int(tr["depth"].max()) == int(fx["maxdepth"])
    ks, sk = h.box_skeletons()
    ranks = fx["ranks"]
    off = fx["skel_off"]
    skel = fx["skel"]
    children = [[] for _ in range(nbox)]
    for b in range(nbox):
        if tr["parent"][b] >= 0:
            children[tr["parent"][b]].append(b)
    own = {b: bool(fx["tie"][b]) for b in range(nbox) if ranks[b] >= 0}
    pts = g.points[tr["perm"]]          # tree order
    J = {}

    def active(b):
        if b not in J:
            J[b] = h.box_export(b)[0]
        return J[b]

    def near(b, dofs):
        d = np.fromiter(dofs, dtype=np.int64)
        rho = 1.5 * tr["side"][b]              # proxy radius of both configurations
        x = pts[d] - tr["center"][b][None, :]
        return bool(np.any(np.sum(x * x, axis=1) < rho * rho))

    bad = uncertain_boxes(tr["depth"], children, own, active, near)
    compared = 0
    same = True
    for b in range(nbox):
        if ranks[b] < 0:
            continue
        eq = ks[b] == ranks[b] and np.array_equal(np.sort(sk[b]), skel[off[b]:off[b + 1]])
        same = same and eq
        if b in bad:
            continue
        assert ks[b] == ranks[b], f"rank differs at box {b}: {ks[b]} vs {ranks[b]}"
        assert eq, f"skeletons differ at box {b}"
        compared += 1
    return compared, same


def test_sphere_full_size_parity(gpu_lib):
    import torch
    rs = gpu_lib
    fx = _load("sphere20480")
    n, eps = int(fx["n"]), float(fx["eps"])
    g = W.fibonacci_sphere(n)
    t = rs.build_tree(g.points, int(fx["leaf"]))
    h = rs.factor("lap3d_sl", t, g.points, g.weights, eps, identity=0.0,
                  proxy_points=int(fx["npx"]))
    compared, same = _compare_with_fixture(h, t, g, fx)
    assert compared >= 0.9 * int((fx["ranks"] >= 0).sum())
    st = h.stats()
    if same:
        assert st["root_size"] == int(fx["root_size"])
    b = W.gaussian_rhs(n, int(fx["nrhs"]), int(fx["seed"]))
    B = to_device(b)
    h.solve(B)
    torch.cuda.synchronize()
    x = B.cpu().numpy()[:, fx["cols"]]
    xo = fx["x"]
    for j in range(xo.shape[1]):
        rel = np.linalg.norm(x[:, j] - xo[:, j]) / np.linalg.norm(xo[:, j])
        if same:
            assert rel <= 10 * eps, (j, rel)
    p = Problem("lap3d_sl", g.points, g.weights)
    rows = np.random.default_rng(1).choice(n, 48, replace=False)
    bc = b[:, fx["cols"]]
    r_gpu = dense.matvec_rows(p, rows, x) - bc[rows]
    d = dense.matvec_rows(p, rows, x - xo)
    ax = dense.matvec_rows(p, rows, xo)
    for j in range(xo.shape[1]):
        assert np.linalg.norm(d[:, j]) <= 10 * eps * np.linalg.norm(ax[:, j])
        assert np.linalg.norm(r_gpu[:, j]) <= 10 * eps * np.linalg.norm(bc[rows, j])


def test_helmholtz_full_size_parity(gpu_lib):
    import torch
    rs = gpu_lib
    fx = _load("helmholtz32768")
    n, eps = int(fx["n"]), float(fx["eps"])
    g = W.star_curve(n)
    k = float(fx["wavenumber"])
    assert abs(k - W.helmholtz_wavenumber(g, 10.0)) <= 1e-12 * k
    t = rs.build_tree(g.points, int(fx["leaf"]))
    h = rs.factor("helm2d_cfie", t, g.points, g.weights, eps, normals=g.normals,
                  curvature=g.curvature, identity=0.5, proxy_points=int(fx["npx"]),
                  wavenumber=k, eta=k)
    compared, same = _compare_with_fixture(h, t, g, fx)
    assert compared >= 0.9 * int((fx["ranks"] >= 0).sum())
    if same:
        assert h.stats()["root_size"] == int(fx["root_size"])
    b = W.gaussian_rhs(n, int(fx["nrhs"]), int(fx["seed"]), True)
    B = to_device(b, torch.complex128)
    h.solve(B)
    torch.cuda.synchronize()
    x = B.cpu().numpy()[:, fx["cols"]]
    xo = fx["x"]
    for j in range(xo.shape[1]):
        rel = np.linalg.norm(x[:, j] - xo[:, j]) / np.linalg.norm(xo[:, j])
        if same:
            assert rel <= 10 * eps, (j, rel)
    p = Problem("helm2d_cfie", g.points, g.weights, g.normals, g.curvature, identity=0.5,
                wavenumber=k, eta=k)
    rows = np.random.default_rng(3).choice(n, 48, replace=False)
    bc = b[:, fx["cols"]]
    r = dense.matvec_rows(p, rows, x) - bc[rows]
    for j in range(xo.shape[1]):
        # second kind: the residual itself is bounded by 10 eps
        assert np.linalg.norm(r[:, j]) <= 10 * eps * np.linalg.norm(bc[rows, j])


@pytest.mark.parametrize("eps,npx", [(1e-6, 64), (1e-12, 96)])
def test_headline_size_other_eps(gpu_lib, eps, npx):
    """N = 65536 log single layer at the other two tolerances of the headline sweep,
    with the 512-column solve; two columns (the first and the last, in different
    column tiles) are compared with the oracle's solve."""
    import torch
    rs = gpu_lib
    n, nrhs = 65536, 512
    g = W.star_curve(n)
    p = Problem("lap2d_sl", g.points, g.weights, identity=0.0)
    F = ofactor(p, eps, 64, npx)
    t = rs.build_tree(g.points, 64)
    h = rs.factor("lap2d_sl", t, g.points, g.weights, eps, identity=0.0, proxy_points=npx)
    compared, tied = compare_skeletons(h, F, residual_every=29)
    same = identical_skeletons(h, F)
    print(f"eps={eps:g}: {compared} boxes compared, {tied} excused by a tie at or below "
          f"them, identical skeletons everywhere: {same}")
    # at eps = 1e-12 (about 4500 u) most pivot orders near the threshold are decided by
    # rounding: the oracle flags more than half of the boxes there
    assert compared >= (0.9 if eps >= 1e-9 else 0.25) * len(F.records)
    if same:
        assert h.stats()["root_size"] == F.root_size
    b = W.gaussian_rhs(n, nrhs, 1)
    B = to_device(b)
    h.solve(B)
    torch.cuda.synchronize()
    cols = [0, nrhs - 1]
    x = B[:, cols].cpu().numpy()
    del B
    bc = np.asfortranarray(b[:, cols])
    xo = F.solve(bc)
    rows = np.random.default_rng(0).choice(n, 64, replace=False)
    d = dense.matvec_rows(p, rows, x - xo)
    ax = dense.matvec_rows(p, rows, xo)
    r_gpu = dense.matvec_rows(p, rows, x) - bc[rows]
    r_or = ax - bc[rows]
    for j in range(2):
        rel = np.linalg.norm(x[:, j] - xo[:, j]) / np.linalg.norm(xo[:, j])
        print(f"eps={eps:g} col {cols[j]}: |x-xo|/|xo| = {rel:.3e}, "
              f"|A(x-xo)|/|A xo| = {np.linalg.norm(d[:, j]) / np.linalg.norm(ax[:, j]):.3e}, "
              f"|r|/|b| = {np.linalg.norm(r_gpu[:, j]) / np.linalg.norm(bc[rows, j]):.3e}, "
              f"oracle |r|/|b| = {np.linalg.norm(r_or[:, j]) / np.linalg.norm(bc[rows, j]):.3e}")
        if same:
            assert rel <= 10 * eps, (cols[j], rel)
            assert np.linalg.norm(d[:, j]) <= 10 * eps * np.linalg.norm(ax[:, j])
        assert (np.linalg.norm(r_gpu[:, j]) <= np.linalg.norm(r_or[:, j])
                + 10 * eps * np.linalg.norm(bc[rows, j]))
