"""Writes the oracle's expected values for the full-size parity tests.

Test infrastructure: calls only the CPU oracle (``oracle/``) and the seeded input
generators (``workloads/``); nothing here touches the device library.  Each fixture is
a NumPy ``.npz`` archive (no pickled objects; load with ``allow_pickle=False``) holding,
for one configuration:

* the tree summary (box count, maximum depth) and the root size;
* per box: rank k (-1 for the root), the skeleton set (tree positions, ascending) and
  a tie flag (a tied pivot step or a rank decision within 1e-10 of the threshold, the
  readings under which skeleton sets are comparable);
* per box: the first and the k-th pivot magnitude |R_00|, |R_{k-1,k-1}| and the next
  one |R_kk| (for the conditioning of R11 and the ID residual bound);
* the oracle's solution x = A_eps^{-1} b for the listed right-hand-side columns
  (b = workloads.gaussian_rhs(n, nrhs, seed)[:, cols]).

Usage (from the repository root; the sphere takes ~15 minutes on 8 cores):

    python tests/golden/make_fixtures.py sphere20480
    python tests/golden/make_fixtures.py helmholtz32768
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import Problem  # noqa: E402
from oracle import factor as ofactor  # noqa: E402

# name -> configuration (geometry, kernel, eps, leaf, proxies, rhs seed/nrhs/columns)
CONFIGS = {
    # unit sphere, N = 20480 Fibonacci points, 3D Laplace single layer, eps = 1e-6,
    # octree leaf 128, 512 proxies on the sphere of radius 1.5 x box side, 64 RHS
    "sphere20480": dict(geom="sphere", n=20480, kind="lap3d_sl", eps=1e-6, leaf=128,
                        npx=512, seed=2, nrhs=64, cols=(0, 1), complex_rhs=False),
    # star curve, N = 32768, exterior combined field 1/2 I + D_k - i k S_k with 10
    # wavelengths across the diameter, eps = 1e-9, leaf 64, 64 proxies
    "helmholtz32768": dict(geom="star", n=32768, kind="helm2d_cfie", eps=1e-9, leaf=64,
                           npx=64, seed=11, nrhs=2, cols=(0,), complex_rhs=True,
                           wavelengths=10.0),
}


def problem(cfg):
    if cfg["geom"] == "sphere":
        g = W.fibonacci_sphere(cfg["n"])
    else:
        g = W.star_curve(cfg["n"])
    if cfg["kind"] == "lap3d_sl":
        return g, Problem("lap3d_sl", g.points, g.weights), {}
    if cfg["kind"] == "helm2d_cfie":
        k = W.helmholtz_wavenumber(g, cfg["wavelengths"])
        return g, Problem("helm2d_cfie", g.points, g.weights, g.normals, g.curvature,
                          identity=0.5, wavenumber=k, eta=k), {"wavenumber": k}
    raise ValueError(cfg["kind"])


def fixture_path(name):
    return os.path.join(HERE, name + ".npz")


def make(name):
    cfg = CONFIGS[name]
    g, p, extra = problem(cfg)
    t0 = time.perf_counter()
    F = ofactor(p, cfg["eps"], cfg["leaf"], cfg["npx"])
    t1 = time.perf_counter()
    t = F.tree
    nb = t.nbox
    ranks = np.full(nb, -1, dtype=np.int32)
    tie = np.zeros(nb, dtype=np.bool_)
    r0 = np.zeros(nb)
    rk1 = np.zeros(nb)
    rk = np.zeros(nb)
    skel_off = np.zeros(nb + 1, dtype=np.int64)
    skel = []
    for b in range(nb):
        r = F.records.get(b)
        if r is not None:
            ranks[b] = r.k
            tie[b] = r.idr.first_tie >= 0 or r.idr.near_threshold
            rd = r.idr.rdiag
            if rd.size:
                r0[b] = rd[0]
                rk1[b] = rd[r.k - 1] if r.k > 0 else 0.0
                rk[b] = rd[r.k] if r.k < rd.size else 0.0
            skel.append(r.skel.astype(np.int64))
            skel_off[b + 1] = skel_off[b] + r.k
        else:
            skel_off[b + 1] = skel_off[b]
    b_all = W.gaussian_rhs(cfg["n"], cfg["nrhs"], cfg["seed"], cfg["complex_rhs"])
    cols = list(cfg["cols"])
    x = F.solve(np.asfortranarray(b_all[:, cols]))
    t2 = time.perf_counter()
    np.savez_compressed(
        fixture_path(name),
        n=cfg["n"], eps=cfg["eps"], leaf=cfg["leaf"], npx=cfg["npx"], seed=cfg["seed"],
        nrhs=cfg["nrhs"], cols=np.array(cols, dtype=np.int32),
        nbox=nb, maxdepth=t.maxdepth, root_size=F.root_size,
        ranks=ranks, tie=tie, rdiag0=r0, rdiag_km1=rk1, rdiag_k=rk,
        skel_off=skel_off, skel=np.concatenate(skel).astype(np.int32) if skel else
        np.zeros(0, dtype=np.int32),
        x=np.ascontiguousarray(x), factor_s=t1 - t0, solve_s=t2 - t1,
        total_skeletons=int(sum(max(0, int(v)) for v in ranks)),
        **extra)
    print(f"{name}: factor {t1 - t0:.1f} s, solve {t2 - t1:.1f} s, boxes {nb}, "
          f"root {F.root_size}, tied boxes {int(tie.sum())}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CONFIGS)
    for nm in names:
        make(nm)
