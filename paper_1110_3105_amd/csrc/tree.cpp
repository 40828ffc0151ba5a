// Quadtree / octree with contiguous index ranges (Section 2.1; the tree rule of the
// experiments in Section 6: uniform subdivision until blocks are small, empty boxes
// truncated).  Host code, compiled with -ffp-contract=off: every coordinate operation
// is a single IEEE operation, so the tree is a deterministic function of the points.
#include "tree.h"

#include <array>

#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "pool.h"

namespace rs {

static constexpr int kMaxDepth = 40;

void Tree::build(int dim_, int64_t n_, const double *pts, int leaf) {
  dim = dim_;
  n = n_;
  leaf_size = leaf;
  double lo[3], hi[3];
  for (int a = 0; a < dim; ++a) {
    lo[a] = pts[a];
    hi[a] = pts[a];
  }
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < dim; ++a) {
      const double v = pts[i * dim + a];
      lo[a] = std::min(lo[a], v);
      hi[a] = std::max(hi[a], v);
    }
  double c0[3] = {0, 0, 0};
  double s0 = 0.0;
  for (int a = 0; a < dim; ++a) {
    c0[a] = (lo[a] + hi[a]) * 0.5;
    s0 = std::max(s0, hi[a] - lo[a]);
  }
  perm.resize(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  center.clear(); side.clear(); depth.clear(); parent.clear(); begin.clear(); end.clear();
  first_child.clear(); nchild.clear(); icoord.clear();

  auto add = [&](const double *c, double s, int d, int p, int64_t b, int64_t e, int code) {
    for (int a = 0; a < 3; ++a)
      icoord.push_back(p < 0 ? 0 : 2 * icoord[3 * p + a] + ((code >> a) & 1));
    for (int a = 0; a < 3; ++a) center.push_back(a < dim ? c[a] : 0.0);
    side.push_back(s);
    depth.push_back(d);
    parent.push_back(p);
    begin.push_back(b);
    end.push_back(e);
    first_child.push_back(-1);
    nchild.push_back(0);
  };
  add(c0, s0, 0, -1, 0, n, 0);
  const int ncode = 1 << dim;
  // Level by level: the boxes of one depth partition their (disjoint) index ranges in
  // parallel, then their children are numbered in box order -- the same breadth-first
  // numbering and stable order as splitting the boxes one after another.
  std::vector<int64_t> tmp(n);
  std::vector<int> code(n);
  std::vector<int> cur = {0};
  while (!cur.empty()) {
    const int nb = (int)cur.size();
    std::vector<std::array<int64_t, 8>> counts(nb);
    std::vector<char> split(nb, 0);
    parallel_for(nb, [&](int bi) {
      const int q = cur[bi];
      const int64_t b = begin[q], e = end[q];
      if (!(e - b > leaf_size && depth[q] < kMaxDepth && side[q] > 0.0)) return;
      split[bi] = 1;
      const double c[3] = {center[3 * q], center[3 * q + 1], center[3 * q + 2]};
      std::array<int64_t, 8> &cnt = counts[bi];
      cnt.fill(0);
      for (int64_t i = b; i < e; ++i) {
        const int64_t g = perm[i];
        int cc = 0;
        for (int a = 0; a < dim; ++a) cc |= (pts[g * dim + a] >= c[a] ? 1 : 0) << a;
        code[i] = cc;
        cnt[cc]++;
      }
      int64_t pos[8];
      int64_t acc = b;
      for (int cc = 0; cc < ncode; ++cc) {
        pos[cc] = acc;
        acc += cnt[cc];
      }
      for (int64_t i = b; i < e; ++i) tmp[pos[code[i]]++] = perm[i];
      std::copy(tmp.begin() + b, tmp.begin() + e, perm.begin() + b);
    }, 1);
    std::vector<int> next;
    for (int bi = 0; bi < nb; ++bi) {
      if (!split[bi]) continue;
      const int q = cur[bi];
      const double c[3] = {center[3 * q], center[3 * q + 1], center[3 * q + 2]};
      const double sq = side[q];
      int64_t off = begin[q];
      for (int cc = 0; cc < ncode; ++cc) {
        const int64_t cnt = counts[bi][cc];
        if (cnt == 0) continue;
        double cch[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) cch[a] = ((cc >> a) & 1) ? c[a] + sq * 0.25 : c[a] - sq * 0.25;
        const int id = (int)side.size();
        if (first_child[q] < 0) first_child[q] = id;
        nchild[q]++;
        add(cch, sq * 0.5, depth[q] + 1, q, off, off + cnt, cc);
        next.push_back(id);
        off += cnt;
      }
    }
    cur.swap(next);
  }
  maxdepth = 0;
  for (int d : depth) maxdepth = std::max(maxdepth, d);
  levels.assign(maxdepth + 1, {});
  for (int bx = 0; bx < (int)side.size(); ++bx) levels[depth[bx]].push_back(bx);
  // tree-order coordinates (structure of arrays)
  coords.assign((size_t)dim * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < dim; ++a) coords[(size_t)a * n + i] = pts[perm[i] * dim + a];
}

}  // namespace rs
