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
  struct Task {
    int bi;
    int64_t i0, i1;
    std::array<int64_t, 8> cnt, pos;
  };
  while (!cur.empty()) {
    const int nb = (int)cur.size();
    std::vector<std::array<int64_t, 8>> counts(nb);
    std::vector<char> split(nb, 0);
    std::vector<Task> tasks;
    for (int bi = 0; bi < nb; ++bi) {
      const int q = cur[bi];
      const int64_t b = begin[q], e = end[q];
      if (!(e - b > leaf_size && depth[q] < kMaxDepth && side[q] > 0.0)) continue;
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
