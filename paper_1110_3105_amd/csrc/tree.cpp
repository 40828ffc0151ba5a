// Quadtree / octree with contiguous index ranges (Section 2.1; the tree rule of the
// experiments in Section 6: uniform subdivision until blocks are small, empty boxes
// truncated).  Host code, compiled with -ffp-contract=off: every coordinate operation
// is a single IEEE operation, so the tree is a deterministic function of the points.
#include "tree.h"

#include <array>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <stdexcept>

#include "pool.h"

namespace rs {

static constexpr int kMaxDepth = 40;

namespace {
// A few large per-point arrays kept between builds (a process builds trees of similar
// sizes again and again).  take() returns a cached array of sufficient capacity, or an
// empty one; give() keeps arrays of at least kMinCached elements, up to kCacheSlots.
constexpr size_t kMinCached = size_t(1) << 14;
constexpr size_t kCacheSlots = 4;
template <class T>
struct BufCache {
  std::mutex mu;
  std::vector<std::vector<T>> bufs;
  std::vector<T> take(size_t n) {
    std::lock_guard<std::mutex> lk(mu);
    for (size_t i = 0; i < bufs.size(); ++i)
      if (bufs[i].capacity() >= n) {
        std::vector<T> v = std::move(bufs[i]);
        bufs.erase(bufs.begin() + (std::ptrdiff_t)i);
        return v;
      }
    return {};
  }
  void give(std::vector<T> &v) {
    if (v.capacity() < kMinCached) return;
    std::lock_guard<std::mutex> lk(mu);
    if (bufs.size() >= kCacheSlots) bufs.erase(bufs.begin());   // keep the newest
    bufs.push_back(std::move(v));
    v = std::vector<T>();
  }
};
template <class T>
BufCache<T> &buf_cache() {
  static BufCache<T> *c = new BufCache<T>();   // never destroyed: trees may outlive main
  return *c;
}
// Sized to n, contents unspecified (every element is written before it is read).
template <class T>
void take_sized(std::vector<T> &v, size_t n) {
  if (v.capacity() < n) {
    std::vector<T> c = buf_cache<T>().take(n);
    if (c.capacity() >= n) v.swap(c);
    buf_cache<T>().give(c);
  }
  v.resize(n);
}
}  // namespace

Tree::~Tree() {
  buf_cache<int64_t>().give(perm);
  buf_cache<double>().give(coords);
}

void Tree::build(int dim_, int64_t n_, const double *pts, int leaf) {
  PlanPool::get().wake();
  dim = dim_;
  n = n_;
  leaf_size = leaf;
  // bounding box: per-chunk extremes, combined in chunk order (min / max are exact)
  constexpr int64_t kPtsChunk = 4096;
  const int nck = (int)std::max<int64_t>(1, (n + kPtsChunk - 1) / kPtsChunk);
  std::vector<std::array<double, 6>> ext(nck);
  parallel_for(nck, [&](int ci) {
    const int64_t i0 = ci * kPtsChunk, i1 = std::min(n, i0 + kPtsChunk);
    std::array<double, 6> &x = ext[ci];
    for (int a = 0; a < dim; ++a) x[a] = x[3 + a] = pts[(i0 < n ? i0 : 0) * dim + a];
    for (int64_t i = i0; i < i1; ++i)
      for (int a = 0; a < dim; ++a) {
        const double v = pts[i * dim + a];
        x[a] = std::min(x[a], v);
        x[3 + a] = std::max(x[3 + a], v);
      }
  }, 1);
  double lo[3], hi[3];
  for (int a = 0; a < dim; ++a) {
    lo[a] = ext[0][a];
    hi[a] = ext[0][3 + a];
    for (int ci = 1; ci < nck; ++ci) {
      lo[a] = std::min(lo[a], ext[ci][a]);
      hi[a] = std::max(hi[a], ext[ci][3 + a]);
    }
  }
  double c0[3] = {0, 0, 0};
  double s0 = 0.0;
  for (int a = 0; a < dim; ++a) {
    c0[a] = (lo[a] + hi[a]) * 0.5;
    s0 = std::max(s0, hi[a] - lo[a]);
  }
  take_sized(perm, (size_t)n);
  parallel_for(nck, [&](int ci) {
    for (int64_t i = ci * kPtsChunk; i < std::min(n, (ci + 1) * kPtsChunk); ++i) perm[i] = i;
  }, 1);
  center.clear(); side.clear(); depth.clear(); parent.clear(); begin.clear(); end.clear();
  first_child.clear(); nchild.clear(); icoord.clear();
  {
    // about two boxes per leaf's worth of points
    const size_t est = (size_t)(2 * n / std::max(1, leaf)) + 64;
    center.reserve(3 * est); icoord.reserve(3 * est); side.reserve(est); depth.reserve(est);
    parent.reserve(est); begin.reserve(est); end.reserve(est); first_child.reserve(est);
    nchild.reserve(est);
  }

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
  std::vector<int64_t> tmp;
  std::vector<int> code;
  take_sized(tmp, (size_t)n);
  take_sized(code, (size_t)n);
  std::vector<int> cur = {0};
  // A box with more than kPartChunk points is partitioned by several tasks (consecutive
  // chunks of its range): each counts its codes, the counts are prefix-summed in chunk
  // order, and each task scatters its points -- the same stable order as one pass.
  constexpr int64_t kPartChunk = 4096;
  constexpr int64_t kSubtreeMax = 4096;
  struct Task {
    int bi;
    int64_t i0, i1;
    std::array<int64_t, 8> cnt, pos;
  };
  auto splits = [&](int64_t b, int64_t e, int d, double sd) {
    return e - b > leaf_size && d < kMaxDepth && sd > 0.0;
  };
  // One subtree per box of roots (those that split), then the merge.
  auto build_subtrees = [&](const std::vector<int> &roots) {
    struct LBox {
      double c[3];
      double s;
      int depth, lparent, code;
      int64_t b, e;
    };
    const int nr = (int)roots.size();
    std::vector<std::vector<LBox>> sub(nr);
    parallel_for(nr, [&](int ri) {
      const int q = roots[ri];
      if (!splits(begin[q], end[q], depth[q], side[q])) return;
      std::vector<LBox> &L = sub[ri];
      LBox r0;
      for (int a = 0; a < 3; ++a) r0.c[a] = center[3 * q + a];
      r0.s = side[q];
      r0.depth = depth[q];
      r0.lparent = -1;
      r0.code = 0;
      r0.b = begin[q];
      r0.e = end[q];
      L.push_back(r0);
      for (size_t li = 0; li < L.size(); ++li) {
        const LBox x = L[li];
        if (!splits(x.b, x.e, x.depth, x.s)) continue;
        int64_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t i = x.b; i < x.e; ++i) {
          const int64_t g = perm[i];
          int cc = 0;
          for (int a = 0; a < dim; ++a) cc |= (pts[g * dim + a] >= x.c[a] ? 1 : 0) << a;
          code[i] = cc;
          cnt[cc]++;
        }
        int64_t pos[8], acc = x.b;
        for (int cc = 0; cc < ncode; ++cc) {
          pos[cc] = acc;
          acc += cnt[cc];
        }
        for (int64_t i = x.b; i < x.e; ++i) tmp[pos[code[i]]++] = perm[i];
        std::copy(tmp.begin() + x.b, tmp.begin() + x.e, perm.begin() + x.b);
        int64_t off = x.b;
        for (int cc = 0; cc < ncode; ++cc) {
          if (cnt[cc] == 0) continue;
          LBox ch;
          for (int a = 0; a < 3; ++a)
            ch.c[a] = a < dim ? (((cc >> a) & 1) ? x.c[a] + x.s * 0.25 : x.c[a] - x.s * 0.25) : 0.0;
          ch.s = x.s * 0.5;
          ch.depth = x.depth + 1;
          ch.lparent = (int)li;
          ch.code = cc;
          ch.b = off;
          ch.e = off + cnt[cc];
          L.push_back(ch);
          off += cnt[cc];
        }
      }
    }, 1);
    // merge: boxes of one depth are consecutive in each subtree's breadth-first list
    std::vector<std::vector<int>> gid(nr);
    std::vector<size_t> at(nr, 1);
    for (int ri = 0; ri < nr; ++ri) {
      gid[ri].assign(sub[ri].size(), -1);
      if (!sub[ri].empty()) gid[ri][0] = roots[ri];
    }
    for (int d = depth[roots[0]] + 1;; ++d) {
      bool any = false;
      for (int ri = 0; ri < nr; ++ri) {
        const std::vector<LBox> &L = sub[ri];
        size_t &li = at[ri];
        for (; li < L.size() && L[li].depth == d; ++li) {
          const LBox &x = L[li];
          const int pg = gid[ri][x.lparent];
          const int id = (int)side.size();
          if (first_child[pg] < 0) first_child[pg] = id;
          nchild[pg]++;
          add(x.c, x.s, d, pg, x.b, x.e, x.code);
          gid[ri][li] = id;
          any = true;
        }
      }
      if (!any) break;
    }
  };
  // The first kTop levels in one pass when the root splits: each point's cell kTop levels
  // down (its quadrant codes along the centers its boxes will have, formed by the same
  // operations as the boxes' own centers), then one stable counting sort by that cell --
  // the order of kTop successive stable partitions.  A box that stops splitting above
  // depth kTop gets its range back in caller order, the order its level left it in.
  constexpr int kTop = 3;
  if (splits(0, n, 0, s0)) {
    const int nbk = 1 << (dim * kTop);
    std::vector<int64_t> hist((size_t)nck * nbk, 0);
    parallel_for(nck, [&](int ci) {
      int64_t *hc = &hist[(size_t)ci * nbk];
      for (int64_t i = ci * kPtsChunk; i < std::min(n, (ci + 1) * kPtsChunk); ++i) {
        const double *x = pts + i * dim;
        double c[3] = {c0[0], c0[1], c0[2]};
        double sq = s0;
        int key = 0;
        for (int l = 0; l < kTop; ++l) {
          int cc = 0;
          for (int a = 0; a < dim; ++a) cc |= (x[a] >= c[a] ? 1 : 0) << a;
          for (int a = 0; a < dim; ++a) c[a] = ((cc >> a) & 1) ? c[a] + sq * 0.25 : c[a] - sq * 0.25;
          sq = sq * 0.5;
          key = (key << dim) | cc;
        }
        code[i] = key;
        hc[key]++;
      }
    }, 1);
    std::vector<int64_t> kcount(nbk + 1, 0);      // kcount[key]: start of the key's run
    {
      int64_t acc = 0;
      for (int key = 0; key < nbk; ++key) {
        kcount[key] = acc;
        for (int ci = 0; ci < nck; ++ci) {
          int64_t &h = hist[(size_t)ci * nbk + key];
          const int64_t c = h;
          h = acc;                                  // the chunk's first slot for the key
          acc += c;
        }
      }
      kcount[nbk] = acc;
    }
    parallel_for(nck, [&](int ci) {
      int64_t *hc = &hist[(size_t)ci * nbk];
      for (int64_t i = ci * kPtsChunk; i < std::min(n, (ci + 1) * kPtsChunk); ++i)
        perm[hc[code[i]]++] = i;
    }, 1);
    // boxes of depths 1..kTop from the runs of the cells (key ranges)
    std::vector<int> lvl = {0};
    std::vector<int> klo = {0};
    for (int l = 1; l <= kTop; ++l) {
      std::vector<int> next, nklo;
      const int span = 1 << (dim * (kTop - l));     // keys per child cell
      for (size_t qi = 0; qi < lvl.size(); ++qi) {
        const int q = lvl[qi];
        if (!splits(begin[q], end[q], depth[q], side[q])) {
          std::sort(perm.begin() + begin[q], perm.begin() + end[q]);
          continue;
        }
        const double c[3] = {center[3 * q], center[3 * q + 1], center[3 * q + 2]};
        const double sq = side[q];
        for (int cc = 0; cc < ncode; ++cc) {
          const int k0 = klo[qi] + cc * span;
          const int64_t b = kcount[k0], e = kcount[k0 + span];
          if (e == b) continue;
          double cch[3] = {0, 0, 0};
          for (int a = 0; a < dim; ++a) cch[a] = ((cc >> a) & 1) ? c[a] + sq * 0.25 : c[a] - sq * 0.25;
          const int id = (int)side.size();
          if (first_child[q] < 0) first_child[q] = id;
          nchild[q]++;
          add(cch, sq * 0.5, depth[q] + 1, q, b, e, cc);
          next.push_back(id);
          nklo.push_back(k0);
        }
      }
      lvl.swap(next);
      klo.swap(nklo);
    }
    cur.swap(lvl);
  }
  while (!cur.empty()) {
    const int nb = (int)cur.size();
    // Once every box still to split holds at most kSubtreeMax points, each of them builds
    // its whole subtree in one task (breadth first, on its own index range), and the
    // subtrees are merged depth by depth in box order -- the numbering and the point
    // order of splitting the levels one after another.
    {
      int nsplit = 0;
      bool small = true;
      for (int q : cur)
        if (splits(begin[q], end[q], depth[q], side[q])) {
          ++nsplit;
          small = small && end[q] - begin[q] <= kSubtreeMax;
        }
      if (nsplit > 0 && small) {
        build_subtrees(cur);
        break;
      }
    }
    std::vector<std::array<int64_t, 8>> counts(nb);
    std::vector<char> split(nb, 0);
    std::vector<Task> tasks;
    for (int bi = 0; bi < nb; ++bi) {
      const int q = cur[bi];
      const int64_t b = begin[q], e = end[q];
      if (!splits(b, e, depth[q], side[q])) continue;
      split[bi] = 1;
      for (int64_t i0 = b; i0 < e; i0 += kPartChunk) {
        Task tk;
        tk.bi = bi;
        tk.i0 = i0;
        tk.i1 = std::min(e, i0 + kPartChunk);
        tasks.push_back(tk);
      }
    }
    const int nt = (int)tasks.size();
    auto count_task = [&](Task &tk) {
      const int q = cur[tk.bi];
      const double c[3] = {center[3 * q], center[3 * q + 1], center[3 * q + 2]};
      tk.cnt.fill(0);
      for (int64_t i = tk.i0; i < tk.i1; ++i) {
        const int64_t g = perm[i];
        int cc = 0;
        for (int a = 0; a < dim; ++a) cc |= (pts[g * dim + a] >= c[a] ? 1 : 0) << a;
        code[i] = cc;
        tk.cnt[cc]++;
      }
    };
    bool one_per_box = true;
    for (int ti = 1; ti < nt; ++ti) one_per_box = one_per_box && tasks[ti].bi != tasks[ti - 1].bi;
    if (one_per_box) {   // every box in one task: count, scatter and copy back in place
      parallel_for(nt, [&](int ti) {
        Task &tk = tasks[ti];
        count_task(tk);
        std::array<int64_t, 8> &cnt = counts[tk.bi];
        cnt = tk.cnt;
        int64_t pos[8], acc = tk.i0;
        for (int cc = 0; cc < ncode; ++cc) {
          pos[cc] = acc;
          acc += cnt[cc];
        }
        for (int64_t i = tk.i0; i < tk.i1; ++i) tmp[pos[code[i]]++] = perm[i];
        std::copy(tmp.begin() + tk.i0, tmp.begin() + tk.i1, perm.begin() + tk.i0);
      }, 1);
    } else {
      parallel_for(nt, [&](int ti) { count_task(tasks[ti]); }, 1);
      for (int ti = 0; ti < nt;) {      // per box: child offsets, then each task's start
        const int bi = tasks[ti].bi;
        int te = ti;
        std::array<int64_t, 8> &cnt = counts[bi];
        cnt.fill(0);
        for (; te < nt && tasks[te].bi == bi; ++te)
          for (int cc = 0; cc < ncode; ++cc) cnt[cc] += tasks[te].cnt[cc];
        int64_t acc = begin[cur[bi]];
        for (int cc = 0; cc < ncode; ++cc) {
          for (int t2 = ti; t2 < te; ++t2) {
            tasks[t2].pos[cc] = acc;
            acc += tasks[t2].cnt[cc];
          }
        }
        ti = te;
      }
      parallel_for(nt, [&](int ti) {
        Task &tk = tasks[ti];
        for (int64_t i = tk.i0; i < tk.i1; ++i) tmp[tk.pos[code[i]]++] = perm[i];
      }, 1);
      parallel_for(nt, [&](int ti) {
        std::copy(tmp.begin() + tasks[ti].i0, tmp.begin() + tasks[ti].i1,
                  perm.begin() + tasks[ti].i0);
      }, 1);
    }
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
  buf_cache<int64_t>().give(tmp);
  buf_cache<int>().give(code);
  // tree-order coordinates (structure of arrays; every entry is written below)
  take_sized(coords, (size_t)dim * n);
  parallel_for(nck, [&](int ci) {
    const int64_t i0 = ci * kPtsChunk, i1 = std::min(n, i0 + kPtsChunk);
    for (int64_t i = i0; i < i1; ++i)
      for (int a = 0; a < dim; ++a) coords[(size_t)a * n + i] = pts[perm[i] * dim + a];
  }, 1);
}

}  // namespace rs
