"""Many-problem batches on the MI355X: shared per-level launches across problems.

A batch of independent problems (different sizes, curves and kernels) is factored and
solved in shared launches; every problem's skeletons and solutions must be bitwise
identical to factoring and solving it alone, and agree with the oracle.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Problem
from oracle import factor as ofactor

pytestmark = pytest.mark.gpu


def _spec(rs, g, kind, eps, leaf, npx):
    t = rs.build_tree(g.points, leaf)
    d = dict(kind=kind, tree=t, points=g.points, weights=g.weights, eps=eps, proxy_points=npx)
    if kind == "lap2d_dl":
        d.update(normals=g.normals, curvature=g.curvature, identity=-0.5)
    return d


def _batch(rs):
    rng = np.random.default_rng(7)
    specs = []
    for n in (1024, 1500, 2500, 777):
        amps = rng.uniform(0, 0.04, 8)
        ph = rng.uniform(0, 2 * np.pi, 8)
        specs.append((W.random_curve(n, amps, ph), "lap2d_dl", 1e-9, 64, 64))
    specs.append((W.star_curve(3000), "lap2d_sl", 1e-9, 64, 64))
    specs.append((W.fibonacci_sphere(1200), "lap3d_sl", 1e-6, 128, 256))
    return [(g, _spec(rs, g, kind, eps, leaf, npx)) for (g, kind, eps, leaf, npx) in specs]


def _solve_alone(h, b):
    import torch
    B = torch.tensor(b.T.copy(), device="cuda").t()
    h.solve(B)
    torch.cuda.synchronize()
    return B.cpu().numpy()


def test_batched_factor_and_solve_bitwise_equal_to_single(gpu_lib):
    import torch
    rs = gpu_lib
    items = _batch(rs)
    hb = rs.factor_batched([s for _, s in items])
    hs = [rs.factor(s["kind"], s["tree"], s["points"], s["weights"], s["eps"],
                    normals=s.get("normals"), curvature=s.get("curvature"),
                    identity=s.get("identity", 0.0), proxy_points=s["proxy_points"])
          for _, s in items]
    for a, b in zip(hb, hs):
        ka, sa = a.box_skeletons()
        kb, sb = b.box_skeletons()
        assert np.array_equal(ka, kb)
        assert all(np.array_equal(x, y) for x, y in zip(sa, sb))
        assert a.stats()["root_size"] == b.stats()["root_size"]
    nrhs = [1, 5, 37, 2, 64, 3]
    rhs = [W.gaussian_rhs(g.n, k, 100 + i) for i, ((g, _), k) in enumerate(zip(items, nrhs))]
    blocks = [torch.tensor(b.T.copy(), device="cuda").t() for b in rhs]
    rs.solve_batched(hb, blocks)
    torch.cuda.synchronize()
    for blk, b, h in zip(blocks, rhs, hs):
        assert np.array_equal(blk.cpu().numpy(), _solve_alone(h, b))


def test_batched_solve_repeated_handle_disjoint_blocks(gpu_lib):
    import torch
    rs = gpu_lib
    g = W.star_curve(2000)
    h = rs.factor("lap2d_sl", rs.build_tree(g.points, 64), g.points, g.weights, 1e-9)
    b = W.gaussian_rhs(2000, 10, 3)
    full = torch.tensor(b.T.copy(), device="cuda").t()
    parts = [full[:, 0:3], full[:, 3:4], full[:, 4:10]]
    rs.solve_batched([h, h, h], parts)
    torch.cuda.synchronize()
    assert np.array_equal(full.cpu().numpy(), _solve_alone(h, b))


def test_batched_matches_oracle(gpu_lib):
    import torch
    rs = gpu_lib
    items = _batch(rs)[:3]
    hb = rs.factor_batched([s for _, s in items])
    for (g, s), h in zip(items, hb):
        p = Problem(s["kind"], g.points, g.weights, s.get("normals"), s.get("curvature"),
                    identity=s.get("identity", 0.0))
        F = ofactor(p, s["eps"], 64, s["proxy_points"])
        ks, sk = h.box_skeletons()
        for bx, rec in F.records.items():
            if rec.idr.first_tie < 0 and not rec.idr.near_threshold:
                assert ks[bx] == rec.k
        b = W.gaussian_rhs(g.n, 2, 9)
        B = torch.tensor(b.T.copy(), device="cuda").t()
        rs.solve_batched([h], [B])
        torch.cuda.synchronize()
        x, xo = B.cpu().numpy(), F.solve(b)
        assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 10 * s["eps"]


def test_batched_argument_errors(gpu_lib):
    import torch
    rs = gpu_lib
    g = W.star_curve(300)
    h = rs.factor("lap2d_sl", rs.build_tree(g.points, 64), g.points, g.weights, 1e-9)
    bad = torch.zeros(299, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        rs.solve_batched([h], [bad])
    with pytest.raises(rs.RSError) as ei:
        rs.factor_batched([dict(kind="lap2d_sl", tree=rs.build_tree(g.points, 64),
                                points=g.points, weights=g.weights, eps=-1.0)])
    assert ei.value.code == 1


def test_many_problem_family_parity_on_16(gpu_lib):
    """Members 0..15 of the benchmark's 256-curve family (N ~ U{1024..16384}, interior
    double layer, eps = 1e-9, leaf 64, 64 proxies), factored in one batch: each against
    its own oracle run (skeletons where no tie reaches a box; the solution to 10 eps when
    all skeletons agree), and its residual against the compressed operator the batch
    inverted (rs_matvec over all rows)."""
    import torch
    from parity_util import compare_skeletons, identical_skeletons, to_device
    rs = gpu_lib
    eps = 1e-9
    fam = [W.random_curve_problem(p) for p in range(16)]
    specs = [_spec(rs, g, "lap2d_dl", eps, 64, 64) for g, _ in fam]
    hb = rs.factor_batched(specs)
    Bs = [to_device(b) for _, b in fam]
    rs.solve_batched(hb, Bs)
    torch.cuda.synchronize()
    for (g, b), h, B in zip(fam, hb, Bs):
        p = Problem("lap2d_dl", g.points, g.weights, g.normals, g.curvature, identity=-0.5)
        F = ofactor(p, eps, 64, 64)
        compared, _ = compare_skeletons(h, F, residual_every=5)
        assert compared >= 0.9 * len(F.records)
        x = B.cpu().numpy()
        if identical_skeletons(h, F):
            xo = F.solve(b)
            assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 10 * eps
        Y = h.matvec(B)
        torch.cuda.synchronize()
        assert np.linalg.norm(Y.cpu().numpy() - b) / np.linalg.norm(b) <= 1e-12
