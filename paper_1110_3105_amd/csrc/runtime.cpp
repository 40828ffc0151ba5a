// Factor and solve drivers.
//
// Factorization (Sections 3.1, 3.2, 3.4) runs level-synchronously from the finest
// depth to the root.  Per step, the host plans every box of the level (active set,
// near DOFs inside the proxy surface), the device assembles and compresses all boxes
// in one launch per kernel, the ranks and skeleton orders come back to the host (they
// decide the next level's active sets), and one more launch forms the diagonal blocks
// and box factors.  Several problems are factored together by aligning them at their
// finest depth: step t handles depth maxdepth_p - t of every problem p.
//
// Host planning is compiled with -ffp-contract=off so that the near-field test
// |x - c|^2 < rho^2 is evaluated with exactly the same roundings as the reference.
#include "runtime.h"
#include "pool.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <condition_variable>
#include <functional>
#include <thread>

namespace rs {

void LevelRec::partition_classes(int mfma_limit) {
  std::vector<int> order(sweep.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  auto small = [&](int i) { return sweep[i].k + sweep[i].r <= mfma_limit; };
  std::stable_partition(order.begin(), order.end(), small);
  std::vector<SweepBox> s2;
  std::vector<int> b2;
  n_small = 0;
  max_n_small = max_n_large = max_k_large = max_r_large = 0;
  for (int i : order) {
    s2.push_back(sweep[i]);
    if (!boxes.empty()) b2.push_back(boxes[i]);
    const int n = sweep[i].k + sweep[i].r;
    if (small(i)) {
      n_small++;
      max_n_small = std::max(max_n_small, n);
    } else {
      max_n_large = std::max(max_n_large, n);
      max_k_large = std::max(max_k_large, (int)sweep[i].k);
      max_r_large = std::max(max_r_large, (int)sweep[i].r);
    }
  }
  sweep.swap(s2);
  if (!boxes.empty()) boxes.swap(b2);
}

namespace {
struct ChunkCache {
  std::mutex mu;
  std::vector<std::unique_ptr<DevBuf>> free;
  size_t bytes = 0;
  // smallest cached chunk of at least `need` bytes, or null
  std::unique_ptr<DevBuf> take(size_t need) {
    std::lock_guard<std::mutex> lk(mu);
    int best = -1;
    for (int i = 0; i < (int)free.size(); ++i)
      if (free[i]->bytes >= need && (best < 0 || free[i]->bytes < free[best]->bytes)) best = i;
    if (best < 0) return nullptr;
    std::unique_ptr<DevBuf> c = std::move(free[best]);
    free.erase(free.begin() + best);
    bytes -= c->bytes;
    return c;
  }
  void give(std::unique_ptr<DevBuf> c) {
    std::lock_guard<std::mutex> lk(mu);
    if (bytes + c->bytes > kChunkCacheBytes) return;      // released by its destructor
    bytes += c->bytes;
    free.push_back(std::move(c));
  }
};
ChunkCache &chunk_cache() {
  static ChunkCache *c = new ChunkCache();   // lives for the process
  return *c;
}
}  // namespace

void Arena::release() {
  for (auto &c : chunks)
    if (c && c->p) chunk_cache().give(std::move(c));
  chunks.clear();
  used = total = 0;
}

Arena::~Arena() { release(); }

void *Arena::alloc(size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  if (chunks.empty() || used + bytes > chunks.back()->bytes) {
    const size_t want = std::max<size_t>(bytes, size_t(8) << 20);
    std::unique_ptr<DevBuf> c = chunk_cache().take(want);
    if (!c) {
      c = std::make_unique<DevBuf>();
      c->ensure(want);
    }
    chunks.push_back(std::move(c));
    used = 0;
  }
  void *p = static_cast<char *>(chunks.back()->p) + used;
  used += bytes;
  total += bytes;
  return p;
}

namespace {

// Pinned host staging (grow-only; a grow waits for the device first).
struct PinnedBuf {
  void *p = nullptr;
  size_t bytes = 0;
  void ensure(size_t b) {
    if (b <= bytes) return;
    RS_HIP_CHECK(hipDeviceSynchronize());
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    RS_HIP_CHECK(hipHostMalloc(&p, b < 256 ? 256 : b, hipHostMallocDefault));
    bytes = b < 256 ? 256 : b;
  }
};

// Transient device buffers shared by all factor calls (grown on demand).  The buffers a
// level's box factorization reads (index pool, skeleton order, ranks, descriptors) come
// in two sets used by alternate levels: the factorization of one level runs on a second
// stream while the next level is compressed.
struct Scratch {
  DevBuf pool, comp, comp_id, fac, M, order, ranks, work, err, probs, partials;
  DevBuf pool2[2], order2[2], ranks2[2], fac2[2];
  PinnedBuf hfac[2];
  // Pinned staging of the factor's host-to-device uploads: stage() hands out space after
  // the previous staging (its copies may still be queued); stage_reset() returns all of
  // it once the stream that carries the copies has been synchronized.  A grow waits for
  // the device first, so queued copies never read freed memory.
  PinnedBuf hup;
  // Pinned readback of a level's ranks and skeleton orders (sized once per call for the
  // largest level, so it never grows while work is queued)
  PinnedBuf hrd;
  size_t hup_used = 0;
  // timing events of the per-level statistics (two per level), created once
  std::vector<hipEvent_t> timing_ev;
  void timing_events(size_t count) {
    while (timing_ev.size() < count) {
      hipEvent_t e = nullptr;
      RS_HIP_CHECK(hipEventCreate(&e));
      timing_ev.push_back(e);
    }
  }
  void *stage(size_t bytes) {
    size_t off = (hup_used + 255) & ~size_t(255);
    if (off + bytes > hup.bytes) {
      hup.ensure(std::max(off + bytes, 2 * hup.bytes));
      off = 0;
    }
    hup_used = off + bytes;
    return static_cast<char *>(hup.p) + off;
  }
  void stage_reset() { hup_used = 0; }
  template <class T>
  void upload(DevBuf &buf, const std::vector<T> &v, hipStream_t st) {
    const size_t bytes = v.size() * sizeof(T);
    buf.ensure(std::max<size_t>(bytes, 8));
    if (!bytes) return;
    void *h = stage(bytes);
    std::memcpy(h, v.data(), bytes);
    RS_HIP_CHECK(hipMemcpyAsync(buf.p, h, bytes, hipMemcpyHostToDevice, st));
  }
  hipStream_t side = nullptr;                 // box factorizations of compressed levels
  hipStream_t aux = nullptr;                  // the direct compression class of a level
  hipStream_t aux2 = nullptr;                 // the small fused boxes of a level
  hipEvent_t ev_comp = nullptr, ev_side = nullptr, ev_diag[2] = {nullptr, nullptr};
  hipEvent_t ev_up = nullptr, ev_aux = nullptr, ev_aux2 = nullptr, ev_wait = nullptr;
  hipEvent_t ev_root_in = nullptr, ev_root_done = nullptr;   // the roots' launches on aux
  hipEvent_t ev_hook = nullptr;               // the caller's interleaved work (side stream)
  void init_streams() {
    if (side) return;
    RS_HIP_CHECK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    RS_HIP_CHECK(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
    RS_HIP_CHECK(hipStreamCreateWithFlags(&aux2, hipStreamNonBlocking));
    for (hipEvent_t *e : {&ev_comp, &ev_side, &ev_diag[0], &ev_diag[1], &ev_up, &ev_aux, &ev_aux2,
                          &ev_wait, &ev_root_in, &ev_root_done, &ev_hook})
      RS_HIP_CHECK(hipEventCreateWithFlags(e, hipEventDisableTiming));
  }
  // Waits for the work queued on st by polling an event: the level loop waits for each
  // level's ranks, and a blocking wait adds the thread's wake-up to every level.
  void wait_stream(hipStream_t st) {
    RS_HIP_CHECK(hipEventRecord(ev_wait, st));
    while (true) {
      const hipError_t e = hipEventQuery(ev_wait);
      if (e == hipSuccess) return;
      if (e != hipErrorNotReady) RS_HIP_CHECK(e);
      __builtin_ia32_pause();
    }
  }
};

std::mutex g_factor_mutex;
Scratch &scratch() {
  static Scratch *s = new Scratch();   // lives for the process
  return *s;
}


struct ProbState {
  const FactorRequest *req = nullptr;
  rs_factor_s *h = nullptr;
  const Tree *t = nullptr;
  int pidx = 0;
  std::vector<std::vector<int32_t>> J, skel;
  // Near-test candidates per box: boxes of its depth within nbr_radius cells (itself
  // excluded) and coarser leaves within Rc cells of each of its ancestors.
  std::vector<std::vector<int32_t>> nbr, coarse;
  int R = 0, Rc = 0;
  int npx = 0;
  bool log_kernel = false;
  bool sketch = false;       // randomized ID: every box compressed through its row sketch
  int oversample = 0;
};

int cheb(const Tree &t, int a, int b) {
  int64_t m = 0;
  for (int x = 0; x < 3; ++x) m = std::max<int64_t>(m, std::abs(t.icoord[3 * a + x] - t.icoord[3 * b + x]));
  return (int)std::min<int64_t>(m, INT32_MAX);
}

// Candidate lists of the near test (Section 3.2), top-down over the depths with no
// hashing: a box's same-depth neighbours within Rl = max(R, Rc) cells are children of
// its parent or of the parent's neighbours (whose list covers the needed ceil(Rl/2)
// cells), and its coarse-leaf candidates are its parent's plus the leaves among the
// parent's neighbours within Rc cells.  R and Rc are the cell radii that contain every
// point within the proxy radius at the box's depth and at each coarser depth.
void plan_neighbors(ProbState &ps) {
  const Tree &t = *ps.t;
  const double ratio = ps.req->k->proxy_ratio;
  ps.R = (int)std::ceil(ratio - 0.5) + 1;
  ps.Rc = (int)std::ceil((ratio - 0.5) * 0.5) + 1;
  const int Rl = std::max(ps.R, ps.Rc);
  const int nb = t.nbox();
  ps.nbr.assign(nb, {});
  ps.coarse.assign(nb, {});
  for (int d = 1; d <= t.maxdepth; ++d) {
    const std::vector<int> &boxes = t.levels[d];
    parallel_for((int)boxes.size(), [&](int bi) {
      const int b = boxes[bi], p = t.parent[b];
      std::vector<int32_t> &out = ps.nbr[b];
      auto children_of = [&](int q) {
        for (int c = t.first_child[q]; c < t.first_child[q] + t.nchild[q]; ++c)
          if (c != b && cheb(t, c, b) <= Rl) out.push_back(c);
      };
      children_of(p);
      for (int q : ps.nbr[p]) children_of(q);
      std::vector<int32_t> &co = ps.coarse[b];
      co = ps.coarse[p];
      for (int q : ps.nbr[p])
        if (t.is_leaf(q) && cheb(t, q, p) <= ps.Rc) co.push_back(q);
    }, 16);
  }
}

// Near DOFs of every box of depth d: active DOFs outside the box's own active set,
// strictly inside the proxy radius (Section 3.2).  The active DOFs at depth d are the
// active sets of the boxes of depth d and the points of coarser leaves; candidates come
// from the lists of plan_neighbors and each is tested with |x - c|^2 < rho^2.  Candidate
// boxes own disjoint, ascending ranges of tree positions, so visiting them by range
// start yields the list in ascending order.
void plan_near(ProbState &ps, int d, std::vector<std::vector<int32_t>> &near) {
  const Tree &t = *ps.t;
  const std::vector<int> &boxes = t.levels[d];
  const int dim = t.dim;
  const double ratio = ps.req->k->proxy_ratio;
  near.assign(boxes.size(), {});
  parallel_for((int)boxes.size(), [&](int bi) {
    const int b = boxes[bi];
    const double *c = &t.center[3 * b];
    const double rho = ratio * t.side[b];
    const double rho2 = rho * rho;
    std::vector<int32_t> &out = near[bi];
    auto test = [&](int32_t g) {
      double d2 = 0.0;
      for (int a = 0; a < dim; ++a) {
        const double df = t.coords[(size_t)a * t.n + g] - c[a];
        d2 += df * df;
      }
      if (d2 < rho2) out.push_back(g);
    };
    thread_local std::vector<int32_t> cand;
    cand.clear();
    for (int q : ps.nbr[b])
      if (cheb(t, q, b) <= ps.R) cand.push_back(q);
    cand.insert(cand.end(), ps.coarse[b].begin(), ps.coarse[b].end());
    std::sort(cand.begin(), cand.end(),
              [&](int32_t x, int32_t y) { return t.begin[x] < t.begin[y]; });
    for (int q : cand) {
      if (t.depth[q] == d) {
        for (int32_t g : ps.J[q]) test(g);
      } else {
        for (int64_t g = t.begin[q]; g < t.end[q]; ++g) test((int32_t)g);
      }
    }
  }, 8);
}

// Copies the geometry of one request to device memory in tree order.
void setup_problem(ProbState &ps, Scratch &S, hipStream_t st) {
  const rs_kernel &k = *ps.req->k;
  const Tree &t = *ps.t;
  rs_factor_s *h = ps.h;
  const int64_t n = t.n;
  const int dim = t.dim;
  h->dim = dim;
  h->n = n;
  h->kind = k.kind;
  h->cplx = k.kind == RS_HELM2D_CFIE || k.kind == RS_HELM3D_SL;
  // points, normals, weights and curvature in tree order, then the permutation, through
  // the pinned staging (no wait: the staging is reused after the stream's next wait)
  const size_t nd = (size_t)n * (2 * dim + 2);
  double *hx = static_cast<double *>(S.stage(nd * sizeof(double) + (size_t)n * sizeof(int64_t)));
  double *hn = hx + (size_t)dim * n;
  double *hw = hn + (size_t)dim * n;
  double *hk = hw + n;
  int64_t *hp = reinterpret_cast<int64_t *>(hx + nd);
  const int64_t chunk = 4096;
  parallel_for((int)((n + chunk - 1) / chunk), [&](int ci) {
    for (int64_t i = ci * chunk; i < std::min<int64_t>(n, (ci + 1) * chunk); ++i) {
      const int64_t g = t.perm[i];
      for (int a = 0; a < dim; ++a) {
        hx[(size_t)a * n + i] = ps.req->points[g * dim + a];
        hn[(size_t)a * n + i] = k.normals ? k.normals[g * dim + a] : 0.0;
      }
      hw[i] = ps.req->weights[g];
      hk[i] = k.curvature ? k.curvature[g] : 0.0;
      hp[i] = g;
    }
  }, 1);
  double *d = h->arena.alloc_n<double>((int64_t)nd);
  RS_HIP_CHECK(hipMemcpyAsync(d, hx, nd * sizeof(double), hipMemcpyHostToDevice, st));
  h->d_perm = h->arena.alloc_n<int64_t>(n);
  RS_HIP_CHECK(hipMemcpyAsync(h->d_perm, hp, n * sizeof(int64_t), hipMemcpyHostToDevice, st));
  ProbDev &P = h->prob;
  std::memset(&P, 0, sizeof(P));
  for (int a = 0; a < dim; ++a) {
    P.x[a] = d + (size_t)a * n;
    P.nrm[a] = k.normals ? d + (size_t)(dim + a) * n : nullptr;
  }
  P.w = d + (size_t)2 * dim * n;
  P.kappa = k.curvature ? d + (size_t)(2 * dim + 1) * n : nullptr;
  P.kind = k.kind;
  P.dim = dim;
  P.c = k.identity;
  P.npx = k.proxy_points;
  P.log_kernel = (k.kind == RS_LAP2D_SL || k.kind == RS_HELM2D_CFIE) ? 1 : 0;
  P.eps = ps.req->eps;
  P.ratio = k.proxy_ratio;
  P.kwave = (k.kind == RS_HELM2D_CFIE || k.kind == RS_HELM3D_SL) ? k.wavenumber : 0.0;
  P.id_mode = k.id_mode;
  P.oversample = k.oversample;
  P.sketch_seed = k.sketch_seed;
  ps.sketch = k.id_mode == RS_ID_SKETCH;
  ps.oversample = k.oversample;
  P.eta = k.kind == RS_HELM2D_CFIE ? k.eta : 0.0;
  ps.npx = k.proxy_points;
  ps.log_kernel = P.log_kernel != 0;
  const int nb = t.nbox();
  ps.J.assign(nb, {});
  ps.skel.assign(nb, {});
  plan_neighbors(ps);
  h->nbox = nb;
  h->box_k.assign(nb, -1);
  h->box_J.assign(nb, {});
  h->box_skel.assign(nb, {});
  h->box_slot.assign(nb, nullptr);
}

struct StepBox {
  ProbState *ps;
  int box;
};

// Gathers a box's active set: its points (leaf) or its children's skeletons.
void gather_J(ProbState &ps, int b) {
  const Tree &t = *ps.t;
  std::vector<int32_t> &J = ps.J[b];
  J.clear();
  if (t.is_leaf(b)) {
    for (int64_t g = t.begin[b]; g < t.end[b]; ++g) J.push_back((int32_t)g);
  } else {
    for (int c = t.first_child[b]; c < t.first_child[b] + t.nchild[b]; ++c)
      J.insert(J.end(), ps.skel[c].begin(), ps.skel[c].end());
  }
}

// Fills the FacBox child fields of box b (children already factored).
void fill_children(ProbState &ps, int b, FacBox &fb) {
  const Tree &t = *ps.t;
  fb.nchild = t.is_leaf(b) ? 0 : t.nchild[b];
  int lo = 0;
  for (int ci = 0; ci < fb.nchild; ++ci) {
    const int c = t.first_child[b] + ci;
    const int kc = ps.h->box_k[c];
    const int nc = (int)ps.J[c].size();
    fb.child_lo[ci] = lo;
    fb.child_k[ci] = kc;
    fb.child_lam[ci] = ps.h->box_slot[c] + slot_L(kc, nc - kc) * (ps.h->cplx ? 2 : 1);
    lo += kc;
  }
}

void check_err(DevBuf &err, hipStream_t st, const std::vector<StepBox> &items, const char *what) {
  int32_t e = -1;
  RS_HIP_CHECK(hipMemcpyAsync(&e, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  RS_HIP_CHECK(hipStreamSynchronize(st));
  if (e >= 0) {
    const StepBox &sb = items[e];
    char buf[256];
    snprintf(buf, sizeof buf, "%s: zero or non-finite pivot at depth %d, box %d%s", what,
             sb.ps->t->depth[sb.box], sb.box, sb.box == 0 ? " (root)" : "");
    throw UserError{RS_ESINGULAR, buf};
  }
}

}  // namespace

namespace {
using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point a) {
  return std::chrono::duration<double, std::milli>(Clock::now() - a).count();
}
}  // namespace

namespace {

// Factors requests that share one scalar type (all real or all complex).
void factor_group(const std::vector<FactorRequest> &reqs, int launch_mode, hipStream_t st,
                  std::vector<rs_factor_s *> &out, const FactorHooks *hooks) {
  auto t0 = std::chrono::steady_clock::now();
  double plan_ms = 0.0, wait_ms = 0.0;
  const int np = (int)reqs.size();
  std::vector<std::unique_ptr<rs_factor_s>> handles(np);
  std::vector<ProbState> ps(np);
  Scratch &S = scratch();
  S.init_streams();
  hipStream_t side = S.side;
  bool diag_pending[2] = {false, false};
  hipEvent_t last_diag = nullptr;      // the latest box factorization on the side stream
  struct SideSync {      // no side- or aux-stream work outlives this call (also on errors)
    hipStream_t s;
    ~SideSync() { (void)hipStreamSynchronize(s); }
  } side_sync{side}, aux_sync{S.aux}, aux2_sync{S.aux2};
  std::vector<ProbDev> probs(np);
  int max_npx = 0, max_depth = 0;
  for (int p = 0; p < np; ++p) {
    handles[p].reset(new rs_factor_s());
    ps[p].req = &reqs[p];
    ps[p].h = handles[p].get();
    ps[p].t = reqs[p].tree;
    ps[p].pidx = p;
    setup_problem(ps[p], S, st);
    probs[p] = handles[p]->prob;
    max_npx = std::max(max_npx, ps[p].npx);
    max_depth = std::max(max_depth, ps[p].t->maxdepth);
  }
  {
    // a level holds at most every box of each problem and, per problem, at most its n
    // active DOFs
    int64_t cap = 0;
    for (int p = 0; p < np; ++p) cap += ps[p].t->nbox() + ps[p].t->n;
    S.hrd.ensure((size_t)std::max<int64_t>(cap, 1) * sizeof(int32_t));
  }
  S.upload(S.probs, probs, st);
  const ProbDev *d_probs = S.probs.as<ProbDev>();
  if (hooks && np == 1 && hooks->begin) {
    RS_HIP_CHECK(hipEventRecord(S.ev_hook, st));
    RS_HIP_CHECK(hipStreamWaitEvent(side, S.ev_hook, 0));
    hooks->begin(handles[0].get(), side);
  }
  const bool cplx = np > 0 && handles[0]->cplx;
  const int es = cplx ? 2 : 1;                 // doubles per scalar
  S.err.ensure(sizeof(int32_t));
  RS_HIP_CHECK(hipMemsetAsync(S.err.p, 0xff, sizeof(int32_t), st));
  const bool per_box = launch_mode == RS_LAUNCH_PER_BOX;
  // per-level statistics: device time of each step's compression (timing events on st)
  // and host planning time; filled into the handles after the final synchronization
  struct StepTiming {
    hipEvent_t a = nullptr, b = nullptr;
    double plan_ms = 0;
  };
  std::vector<StepTiming> step_t(max_depth + 1);
  S.timing_events(2 * (max_depth + 1));      // kept by the scratch and reused
  auto level_entry = [&](rs_factor_s *h, int depth) -> rs_level_stats & {
    for (rs_level_stats &e : h->level_stats)
      if (e.depth == depth) return e;
    h->level_stats.emplace_back();
    rs_level_stats &e = h->level_stats.back();
    std::memset(&e, 0, sizeof(e));
    e.depth = depth;
    return e;
  };
  int64_t max_m_seen = 0;
  // Every factored box gets a global index; a singular pivot reports the first one,
  // checked once after the root (no host wait per level).
  std::vector<StepBox> all_items;
  // A level's solve data (index lists, sweep descriptors) is not needed to plan the next
  // level, so it is built while the next level compresses (`deferred`).  Host arrays of
  // its uploads stay in `keep_alive` until the next synchronization of the stream.
  struct Deferred {
    std::vector<StepBox> items;
    std::vector<CompBox> comp;
    std::vector<int32_t> ranks, order;
    bool pending = false;
  } dfr;
  std::vector<std::vector<int32_t>> keep_alive;
  auto run_deferred = [&]() {
    if (!dfr.pending) return;
    dfr.pending = false;
    const std::vector<StepBox> &items = dfr.items;
    const std::vector<CompBox> &comp = dfr.comp;
    const std::vector<int32_t> &ranks = dfr.ranks, &order = dfr.order;
    const int cnt = (int)items.size();
    // persistent solve data: index lists (skeletons then redundant, tree positions),
    // one contiguous block and one upload per problem and level
    std::vector<std::vector<int32_t>> idx_keep(np);
    std::vector<int32_t *> d_idx_base(np, nullptr);
    std::vector<int64_t> idx_fill(np, 0);
    for (int i = 0; i < cnt; ++i) idx_fill[items[i].ps->pidx] += comp[i].n;
    for (int p = 0; p < np; ++p) {
      if (idx_fill[p] == 0) continue;
      d_idx_base[p] = ps[p].h->arena.alloc_n<int32_t>(idx_fill[p]);
      idx_keep[p].resize(idx_fill[p]);
      idx_fill[p] = 0;
    }
    std::vector<int64_t> idx_at(cnt);
    for (int i = 0; i < cnt; ++i) {
      const int pi = items[i].ps->pidx;
      idx_at[i] = idx_fill[pi];
      idx_fill[pi] += comp[i].n;
    }
    parallel_for(cnt, [&](int i) {
      ProbState &P = *items[i].ps;
      const int32_t *ord = order.data() + comp[i].order_off;
      int32_t *idx = idx_keep[P.pidx].data() + idx_at[i];
      const std::vector<int32_t> &J = P.J[items[i].box];
      for (int a = 0; a < comp[i].n; ++a) idx[a] = J[ord[a]];
    }, 64);
    for (int i = 0; i < cnt; ++i) {
      ProbState &P = *items[i].ps;
      const int b = items[i].box;
      const int k = ranks[i], n = comp[i].n;
      int32_t *d_idx = d_idx_base[P.pidx] + idx_at[i];
      SweepBox sb;
      sb.k = k;
      sb.r = n - k;
      sb.idx = d_idx;
      double *slot = comp[i].T;
      sb.T = slot + slot_T(k, n - k) * es;
      sb.G = slot + slot_G(k, n - k) * es;
      sb.E = slot + slot_E(k, n - k) * es;
      sb.F = slot + slot_F(k, n - k) * es;
      rs_factor_s *h = P.h;
      const int d = P.t->depth[b];
      if (h->levels.empty() || h->levels.back().depth != d) {
        h->levels.emplace_back();
        h->levels.back().depth = d;
      }
      LevelRec &lv = h->levels.back();
      lv.boxes.push_back(b);
      lv.sweep.push_back(sb);
      lv.max_n = std::max(lv.max_n, n);
      h->stats.total_skeletons += k;
      h->stats.factor_doubles += (slot_size(k, n - k) - (int64_t)k * k) * es;
      h->stats.max_box_n = std::max<int64_t>(h->stats.max_box_n, n);
      h->stats.max_box_m = std::max<int64_t>(h->stats.max_box_m, comp[i].m);
      rs_level_stats &ls = level_entry(h, d);
      ls.boxes++;
      ls.n_total += n;
      ls.k_total += k;
      ls.max_n = std::max(ls.max_n, n);
      ls.max_m = std::max(ls.max_m, (int32_t)comp[i].m);
      ls.factor_doubles += (slot_size(k, n - k) - (int64_t)k * k) * es;
    }
    for (int p = 0; p < np; ++p)
      if (!idx_keep[p].empty()) {
        RS_HIP_CHECK(hipMemcpyAsync(d_idx_base[p], idx_keep[p].data(),
                                    idx_keep[p].size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                    st));
        keep_alive.push_back(std::move(idx_keep[p]));
      }
    // a step holds every box of one depth of each problem in it: those levels are
    // complete, and their sweep descriptors go to the device now (the handle keeps the
    // host copies)
    std::vector<char> stepped(np, 0);
    for (int i = 0; i < cnt; ++i) stepped[items[i].ps->pidx] = 1;
    for (int p = 0; p < np; ++p) {
      if (!stepped[p]) continue;
      rs_factor_s *h = ps[p].h;
      LevelRec &lv = h->levels.back();
      lv.partition_classes(mfma_max_n(cplx));
      lv.d_sweep = h->arena.alloc_n<SweepBox>((int64_t)lv.sweep.size());
      RS_HIP_CHECK(hipMemcpyAsync(lv.d_sweep, lv.sweep.data(), lv.sweep.size() * sizeof(SweepBox),
                                  hipMemcpyHostToDevice, st));
      if (hooks && np == 1 && hooks->level) {   // behind the uploads and the level's factors
        RS_HIP_CHECK(hipEventRecord(S.ev_hook, st));
        RS_HIP_CHECK(hipStreamWaitEvent(side, S.ev_hook, 0));
        hooks->level(h, lv, side);
      }
    }
  };

  // ---- compressed levels, aligned at the finest depth of every problem
  for (int step = 0; step < max_depth; ++step) {
    std::vector<StepBox> items;
    for (int p = 0; p < np; ++p) {
      const int d = ps[p].t->maxdepth - step;
      if (d < 1) continue;
      for (int b : ps[p].t->levels[d]) items.push_back({&ps[p], b});
    }
    if (items.empty()) continue;
    const int cnt = (int)items.size();
    auto tp = Clock::now();
    // plan: active sets and near lists
    std::vector<std::vector<int32_t>> near_all(cnt);
    {
      int idx = 0;
      for (int p = 0; p < np; ++p) {
        const int d = ps[p].t->maxdepth - step;
        if (d < 1) continue;
        const std::vector<int> &lvb = ps[p].t->levels[d];
        parallel_for((int)lvb.size(), [&](int i) { gather_J(ps[p], lvb[i]); }, 64);
        std::vector<std::vector<int32_t>> nr;
        plan_near(ps[p], d, nr);
        for (auto &v : nr) near_all[idx++] = std::move(v);
      }
    }
    // boxes of the fused (register-resident) compression class first -- the ones that
    // fit the 256-thread variants, then the others -- then the split class (registers of
    // two workgroups), then the direct class, so that each class is one contiguous range
    // of the launch (stable order)
    int nf = 0, nfs = 0, nsp = 0;
    {
      std::vector<char> fz(cnt);
      for (int i = 0; i < cnt; ++i) {
        const ProbState &P = *items[i].ps;
        const int n = (int)P.J[items[i].box].size();
        const int m = 2 * (int)near_all[i].size() + 2 * P.npx + (P.log_kernel ? 2 : 0);
        fz[i] = P.sketch ? 0
                : fused_class(cplx, n, m) ? (fused_small(n, m) ? 2 : 1)
                : split_class(cplx, n, m) ? 3 : 0;
        nf += fz[i] == 1 || fz[i] == 2;
        nfs += fz[i] == 2;
        nsp += fz[i] == 3;
      }
      // Within the 512-thread fused class (one workgroup per CU, several rounds per
      // launch on wide levels) the largest blocks go first, so that the last round holds
      // short boxes; a box's arithmetic does not depend on its place in the launch.
      std::vector<int64_t> cost(cnt);
      for (int i = 0; i < cnt; ++i) {
        const ProbState &P = *items[i].ps;
        const int64_t n = (int64_t)P.J[items[i].box].size();
        cost[i] = n * (2 * (int64_t)near_all[i].size() + 2 * P.npx);
      }
      std::vector<StepBox> it2;
      std::vector<std::vector<int32_t>> nr2;
      it2.reserve(cnt);
      nr2.reserve(cnt);
      for (int pass : {2, 1, 3, 0}) {
        std::vector<int> sel;
        for (int i = 0; i < cnt; ++i)
          if (fz[i] == pass) sel.push_back(i);
        if (pass == 1)
          std::stable_sort(sel.begin(), sel.end(),
                           [&](int x, int y) { return cost[x] > cost[y]; });
        for (int i : sel) {
          it2.push_back(items[i]);
          nr2.push_back(std::move(near_all[i]));
        }
      }
      items.swap(it2);
      near_all.swap(nr2);
    }
    const int nd0 = nf + nsp;        // first box of the direct class
    std::vector<CompBox> comp(cnt);
    int64_t M_total = 0, order_total = 0, work_total = 0, pool_total = 0;
    int max_n = 0, max_m_step = 0;
    int max_n_f = 0, max_m_f = 0, max_n_s = 0, max_m_s = 0, max_n_d = 0, max_m_d = 0;
    int max_n_sp = 0, max_m_sp = 0;
    for (int i = 0; i < cnt; ++i) {
      ProbState &P = *items[i].ps;
      const int b = items[i].box;
      CompBox &cb = comp[i];
      std::memset(&cb, 0, sizeof(cb));
      const std::vector<int32_t> &J = P.J[b];
      cb.prob = P.pidx;
      cb.n = (int)J.size();
      cb.nn = (int)near_all[i].size();
      cb.m = 2 * cb.nn + 2 * P.npx + (P.log_kernel ? 2 : 0);
      cb.J_off = pool_total;
      cb.N_off = pool_total + cb.n;
      pool_total += cb.n + cb.nn;
      cb.M_off = M_total;
      // fused and split boxes keep their block in registers and LDS: no arena space
      if (i >= nd0) M_total += (int64_t)cb.m * cb.n;
      if (i < nfs) {
        max_n_s = std::max(max_n_s, cb.n);
        max_m_s = std::max(max_m_s, cb.m);
      } else if (i < nf) {
        max_n_f = std::max(max_n_f, cb.n);
        max_m_f = std::max(max_m_f, cb.m);
      } else if (i < nd0) {
        max_n_sp = std::max(max_n_sp, cb.n);
        max_m_sp = std::max(max_m_sp, cb.m);
      } else {
        max_n_d = std::max(max_n_d, cb.n);
        max_m_d = std::max(max_m_d, cb.m);
      }
      for (int a = 0; a < 3; ++a) cb.cen[a] = P.t->center[3 * b + a];
      cb.rho = P.req->k->proxy_ratio * P.t->side[b];
      cb.order_off = order_total;
      order_total += cb.n;
      cb.kslot = i;
      cb.box = b;
      double *slot = P.h->arena.alloc_n<double>(slot_bound(cb.n) * es);
      cb.T = slot;
      P.h->box_slot[b] = slot;
      work_total += (int64_t)diag_work_elems(cb.n);
      max_n = std::max(max_n, cb.n);
      max_m_step = std::max(max_m_step, cb.m);
      max_m_seen = std::max<int64_t>(max_m_seen, cb.m);
    }
    // randomized ID: the direct-class boxes of sketching problems are compressed through
    // Y = Omega M (ell = min(m, n + oversample) rows) placed after the blocks in the arena
    std::vector<CompBox> comp_id;
    int max_m_id = max_m_d, max_sketch_tiles = 0;
    bool any_sketch = false;
    for (int i = nd0; i < cnt; ++i) any_sketch = any_sketch || items[i].ps->sketch;
    if (any_sketch) {
      comp_id = comp;
      max_m_id = 0;
      for (int i = nd0; i < cnt; ++i) {
        CompBox &ci = comp_id[i];
        const ProbState &P = *items[i].ps;
        const int ell = P.sketch ? std::min<int64_t>(ci.m, (int64_t)ci.n + P.oversample) : ci.m;
        if (ell < ci.m) {
          ci.m = ell;
          ci.M_off = M_total;
          M_total += (int64_t)ell * ci.n;
          max_sketch_tiles = std::max(max_sketch_tiles, ((ell + 15) / 16) * ((ci.n + 15) / 16));
        }
        max_m_id = std::max(max_m_id, ci.m);
      }
    }
    std::vector<int32_t> pool(pool_total);
    parallel_for(cnt, [&](int i) {
      const std::vector<int32_t> &J = items[i].ps->J[items[i].box];
      std::copy(J.begin(), J.end(), pool.begin() + comp[i].J_off);
      std::copy(near_all[i].begin(), near_all[i].end(), pool.begin() + comp[i].N_off);
    }, 64);
    plan_ms += ms_since(tp);
    step_t[step].plan_ms += ms_since(tp);
    if (cpqr_lds_bytes(cplx, max_n, 1 << 30) > 160 * 1024)
      throw UserError{RS_ENOTSUP, "a box's active set exceeds the on-chip ID limit"};
    // this level's buffer set was last read by the box factorization two levels back
    const int par = step & 1;
    DevBuf &Dpool = S.pool2[par], &Dorder = S.order2[par], &Dranks = S.ranks2[par];
    DevBuf &Dfac = S.fac2[par];
    if (diag_pending[par]) RS_HIP_CHECK(hipStreamWaitEvent(st, S.ev_diag[par], 0));
    S.upload(Dpool, pool, st);
    S.upload(S.comp, comp, st);
    if (any_sketch) S.upload(S.comp_id, comp_id, st);
    S.M.ensure(std::max<int64_t>(M_total, 1) * sizeof(double) * es);
    Dorder.ensure(std::max<int64_t>(order_total, 1) * sizeof(int32_t));
    Dranks.ensure(std::max(cnt, 1) * sizeof(int32_t));
    S.work.ensure(std::max<int64_t>(work_total, 1) * sizeof(double) * es);
    S.partials.ensure((size_t)std::max(cnt - nd0, 1) * assemble_chunks(max_n_d, max_m_d) *
                      sizeof(double));
    const CompBox *d_comp = S.comp.as<CompBox>();
    const CompBox *d_comp_id = any_sketch ? S.comp_id.as<CompBox>() : d_comp;
    step_t[step].a = S.timing_ev[2 * step];
    step_t[step].b = S.timing_ev[2 * step + 1];
    RS_HIP_CHECK(hipEventRecord(step_t[step].a, st));
    if (per_box) {
      for (int i = 0; i < cnt; ++i) {
        if (i < nf) {
          ProfScope ps_(RS_K_ID, st);
          launch_compress_fused(d_comp, i, 1, d_probs, Dpool.as<int32_t>(), Dorder.as<int32_t>(),
                                Dranks.as<int32_t>(), comp[i].n, comp[i].m, max_npx, st);
          continue;
        }
        if (i < nd0) {
          ProfScope ps_(RS_K_ID, st);
          launch_compress_split(d_comp, i, 1, d_probs, Dpool.as<int32_t>(), Dorder.as<int32_t>(),
                                Dranks.as<int32_t>(), comp[i].n, comp[i].m, max_npx, st);
          continue;
        }
        {
          ProfScope ps_(RS_K_ASSEMBLE, st);
          launch_assemble(cplx, d_comp, i, 1, d_probs, Dpool.as<int32_t>(), S.M.as<double>(),
                          max_npx, comp[i].n, comp[i].m, S.partials.as<double>(), st);
        }
        ProfScope ps_(RS_K_ID, st);
        if (any_sketch)
          launch_sketch(cplx, d_comp, d_comp_id, i, 1, d_probs, S.M.as<double>(),
                        ((comp_id[i].m + 15) / 16) * ((comp_id[i].n + 15) / 16), st);
        launch_cpqr_id(cplx, d_comp_id, i, 1, d_probs, S.M.as<double>(), Dorder.as<int32_t>(),
                       Dranks.as<int32_t>(), comp[i].n, any_sketch ? comp_id[i].m : comp[i].m,
                       st);
      }
    } else {
      // the classes touch disjoint boxes: with more than one present, the small fused
      // boxes and the split and direct classes run on auxiliary streams beside the other
      // fused boxes
      const int nclass = (nfs > 0) + (nf > nfs) + (nf < cnt);
      const bool both = nclass > 1;
      hipStream_t dst = both ? S.aux : st, sst = both ? S.aux2 : st;
      if (both) {
        RS_HIP_CHECK(hipEventRecord(S.ev_up, st));
        RS_HIP_CHECK(hipStreamWaitEvent(S.aux, S.ev_up, 0));
        RS_HIP_CHECK(hipStreamWaitEvent(S.aux2, S.ev_up, 0));
      }
      if (nfs > 0) {
        ProfScope ps_(RS_K_ID, sst);
        launch_compress_fused(d_comp, 0, nfs, d_probs, Dpool.as<int32_t>(), Dorder.as<int32_t>(),
                              Dranks.as<int32_t>(), max_n_s, max_m_s, max_npx, sst);
      }
      if (nf > nfs) {
        ProfScope ps_(RS_K_ID, st);
        launch_compress_fused(d_comp, nfs, nf - nfs, d_probs, Dpool.as<int32_t>(),
                              Dorder.as<int32_t>(), Dranks.as<int32_t>(), max_n_f, max_m_f,
                              max_npx, st);
      }
      if (nsp > 0) {
        ProfScope ps_(RS_K_ID, dst);
        launch_compress_split(d_comp, nf, nsp, d_probs, Dpool.as<int32_t>(), Dorder.as<int32_t>(),
                              Dranks.as<int32_t>(), max_n_sp, max_m_sp, max_npx, dst);
      }
      if (nd0 < cnt) {
        {
          ProfScope ps_(RS_K_ASSEMBLE, dst);
          launch_assemble(cplx, d_comp, nd0, cnt - nd0, d_probs, Dpool.as<int32_t>(),
                          S.M.as<double>(), max_npx, max_n_d, max_m_d, S.partials.as<double>(),
                          dst);
        }
        ProfScope ps_(RS_K_ID, dst);
        if (any_sketch)
          launch_sketch(cplx, d_comp, d_comp_id, nd0, cnt - nd0, d_probs, S.M.as<double>(),
                        max_sketch_tiles, dst);
        launch_cpqr_id(cplx, d_comp_id, nd0, cnt - nd0, d_probs, S.M.as<double>(),
                       Dorder.as<int32_t>(), Dranks.as<int32_t>(), max_n_d, max_m_id, dst);
      }
      if (both) {
        RS_HIP_CHECK(hipEventRecord(S.ev_aux, S.aux));
        RS_HIP_CHECK(hipStreamWaitEvent(st, S.ev_aux, 0));
        RS_HIP_CHECK(hipEventRecord(S.ev_aux2, S.aux2));
        RS_HIP_CHECK(hipStreamWaitEvent(st, S.ev_aux2, 0));
      }
    }
    RS_HIP_CHECK(hipEventRecord(step_t[step].b, st));
    RS_HIP_CHECK(hipEventRecord(S.ev_comp, st));   // ranks, order and pool of this level
    // The box factorizations need this level's ranks and orders only on the device (the
    // kernel reads them by slot), so their descriptors are built now and the launch is
    // queued on the side stream behind the compression, before the host waits for it.
    const int err_base = (int)all_items.size();
    all_items.insert(all_items.end(), items.begin(), items.end());
    std::vector<FacBox> fac(cnt);
    int64_t woff = 0;
    for (int i = 0; i < cnt; ++i) {
      ProbState &P = *items[i].ps;
      const int b = items[i].box;
      const CompBox &cb = comp[i];
      FacBox &fb = fac[i];
      std::memset(&fb, 0, sizeof(fb));
      fb.prob = P.pidx;
      fb.n = cb.n;
      fb.kslot = i;
      fb.force_k0 = 0;
      fb.leaf = P.t->is_leaf(b) ? 1 : 0;
      fb.J_off = cb.J_off;
      fb.order_off = cb.order_off;
      fb.slot = cb.T;
      fb.work_off = woff;
      woff += (int64_t)diag_work_elems(cb.n);
      fill_children(P, b, fb);
    }
    // descriptors through pinned staging (its previous user, two levels back, is done)
    if (diag_pending[par]) RS_HIP_CHECK(hipEventSynchronize(S.ev_diag[par]));
    const size_t fac_bytes = fac.size() * sizeof(FacBox);
    S.hfac[par].ensure(fac_bytes);
    Dfac.ensure(fac_bytes);
    std::memcpy(S.hfac[par].p, fac.data(), fac_bytes);
    RS_HIP_CHECK(hipStreamWaitEvent(side, S.ev_comp, 0));
    RS_HIP_CHECK(hipMemcpyAsync(Dfac.p, S.hfac[par].p, fac_bytes, hipMemcpyHostToDevice, side));
    const FacBox *d_fac = Dfac.as<FacBox>();
    if (per_box) {
      for (int i = 0; i < cnt; ++i) {
        ProfScope ps_(RS_K_FACTOR, side);
        launch_diag_factor(cplx, d_fac, i, 1, d_probs, Dpool.as<int32_t>(), Dorder.as<int32_t>(),
                           Dranks.as<int32_t>(), S.work.as<double>(), S.err.as<int32_t>(),
                           err_base, comp[i].n, side);
      }
    } else {
      ProfScope ps_(RS_K_FACTOR, side);
      launch_diag_factor(cplx, d_fac, 0, cnt, d_probs, Dpool.as<int32_t>(), Dorder.as<int32_t>(),
                         Dranks.as<int32_t>(), S.work.as<double>(), S.err.as<int32_t>(),
                         err_base, max_n, side);
    }
    RS_HIP_CHECK(hipEventRecord(S.ev_diag[par], side));
    diag_pending[par] = true;
    last_diag = S.ev_diag[par];
    run_deferred();        // the previous level's solve data, while this level compresses
    if ((size_t)(cnt + order_total) * sizeof(int32_t) > S.hrd.bytes)
      throw DeviceError("rank readback exceeds its staging", hipErrorInvalidValue);
    int32_t *hrd = static_cast<int32_t *>(S.hrd.p);
    RS_HIP_CHECK(hipMemcpyAsync(hrd, Dranks.p, cnt * sizeof(int32_t), hipMemcpyDeviceToHost,
                                st));
    if (order_total)
      RS_HIP_CHECK(hipMemcpyAsync(hrd + cnt, Dorder.p, order_total * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, st));
    {
      auto tw = Clock::now();
      S.wait_stream(st);
      wait_ms += ms_since(tw);
    }
    std::vector<int32_t> ranks(hrd, hrd + cnt), order(hrd + cnt, hrd + cnt + order_total);
    S.stage_reset();
    keep_alive.clear();            // the uploads queued before this wait have completed
    auto tp2 = Clock::now();
    for (int i = 0; i < cnt; ++i)
      if (ranks[i] < 0 || ranks[i] > comp[i].n)
        throw DeviceError("interpolative decomposition did not complete (a multi-workgroup "
                          "barrier exceeded its wait limit)", hipErrorLaunchTimeOut);
    // skeleton lists (the next level's active sets) and profiler work counts
    Work w_asm, w_id, w_fac;
    for (int i = 0; i < cnt; ++i) {
      const CompBox &cb = comp[i];
      const int k = ranks[i];
      items[i].ps->h->box_k[items[i].box] = k;
      if (i < nd0) {
        w_id += work_fused(cb.m, cb.n, k);
      } else {
        w_asm += work_assemble(cb.m, cb.n, cplx);
        const int ell = any_sketch ? comp_id[i].m : cb.m;
        w_id += work_id(ell, cb.n, k, cplx);
        if (ell < cb.m) w_id.flops += 2.0 * ell * cb.m * cb.n * (cplx ? 2.0 : 1.0);
      }
      w_fac += work_factor(cb.n, k, cplx);
    }
    parallel_for(cnt, [&](int i) {
      ProbState &P = *items[i].ps;
      const int b = items[i].box;
      const std::vector<int32_t> &J = P.J[b];
      const int32_t *ord = order.data() + comp[i].order_off;
      std::vector<int32_t> &sk = P.skel[b];
      sk.resize(ranks[i]);
      for (int a = 0; a < ranks[i]; ++a) sk[a] = J[ord[a]];
    }, 64);
    prof_add_work(RS_K_ASSEMBLE, w_asm);
    prof_add_work(RS_K_ID, w_id);
    prof_add_work(RS_K_FACTOR, w_fac);
    dfr.items = std::move(items);
    dfr.comp = std::move(comp);
    dfr.ranks = std::move(ranks);
    dfr.order = std::move(order);
    dfr.pending = true;
    plan_ms += ms_since(tp2);
    step_t[step].plan_ms += ms_since(tp2);
  }

  run_deferred();
  // ---- roots: the dense block of the surviving skeletons, fully eliminated (on st,
  // after every box factorization of the side stream: the last one's event covers the
  // earlier ones, and not the solve's upward sweeps a caller may have queued behind it)
  if (last_diag) {
    RS_HIP_CHECK(hipStreamWaitEvent(st, last_diag, 0));
  } else {
    RS_HIP_CHECK(hipEventRecord(S.ev_side, side));
    RS_HIP_CHECK(hipStreamWaitEvent(st, S.ev_side, 0));
  }
  {
    std::vector<StepBox> items;
    std::vector<int32_t> pool;
    std::vector<FacBox> fac;
    int64_t woff = 0;
    int max_n = 0;
    for (int p = 0; p < np; ++p) {
      ProbState &P = ps[p];
      const int b = 0;
      gather_J(P, b);
      const std::vector<int32_t> &J = P.J[b];
      FacBox fb;
      std::memset(&fb, 0, sizeof(fb));
      fb.prob = P.pidx;
      fb.n = (int)J.size();
      fb.force_k0 = 1;
      fb.leaf = P.t->is_leaf(b) ? 1 : 0;
      fb.J_off = (int64_t)pool.size();
      pool.insert(pool.end(), J.begin(), J.end());
      fb.slot = P.h->arena.alloc_n<double>(std::max<int64_t>((int64_t)fb.n * fb.n, 1) * es);
      fb.work_off = woff;
      woff += (int64_t)diag_work_elems(fb.n);
      fill_children(P, b, fb);
      fac.push_back(fb);
      items.push_back({&P, b});
      max_n = std::max(max_n, fb.n);
      P.h->box_k[b] = -1;
      P.h->box_J[b] = J;
      P.h->box_slot[b] = fb.slot;
    }
    S.upload(S.pool, pool, st);
    S.upload(S.fac, fac, st);
    S.work.ensure(std::max<int64_t>(woff, 1) * sizeof(double) * es);
    const FacBox *d_fac = S.fac.as<FacBox>();
    const int err_base = (int)all_items.size();
    all_items.insert(all_items.end(), items.begin(), items.end());
    {
      Work w;
      for (const FacBox &f : fac) w += work_factor(f.n, 0, cplx);
      prof_add_work(RS_K_FACTOR, w);
    }
    // The roots run on the aux stream (after everything queued on st so far), so that
    // work that does not need them -- a solve's permutation and upward sweeps through the
    // compressed levels, when the caller asks for one -- can proceed on st meanwhile.
    const hipStream_t rst = S.aux;
    RS_HIP_CHECK(hipEventRecord(S.ev_root_in, st));
    RS_HIP_CHECK(hipStreamWaitEvent(rst, S.ev_root_in, 0));
    step_t[max_depth].a = S.timing_ev[2 * max_depth];
    step_t[max_depth].b = S.timing_ev[2 * max_depth + 1];
    RS_HIP_CHECK(hipEventRecord(step_t[max_depth].a, rst));
    // roots below the register and wide classes: one workgroup each (k_diag_factor skips
    // the others)
    auto narrow = [&](int n) { return n < kWideRootMinN && !root_in_regs(cplx, n); };
    int max_n_narrow = 0;
    for (const FacBox &f : fac)
      if (narrow(f.n)) max_n_narrow = std::max(max_n_narrow, f.n);
    if (per_box) {
      for (int i = 0; i < np; ++i) {
        if (!narrow(fac[i].n)) continue;
        ProfScope ps_(RS_K_FACTOR, rst);
        launch_diag_factor(cplx, d_fac, i, 1, d_probs, S.pool.as<int32_t>(), nullptr, nullptr,
                           S.work.as<double>(), S.err.as<int32_t>(), err_base, fac[i].n, rst);
      }
    } else if (max_n_narrow > 0) {
      ProfScope ps_(RS_K_FACTOR, rst);
      launch_diag_factor(cplx, d_fac, 0, np, d_probs, S.pool.as<int32_t>(), nullptr, nullptr,
                         S.work.as<double>(), S.err.as<int32_t>(), err_base, max_n_narrow, rst);
    }
    for (int i = 0; i < np; ++i) {
      if (!root_in_regs(cplx, fac[i].n)) continue;
      ProfScope ps_(RS_K_FACTOR, rst);
      launch_root_regs(d_fac + i, fac[i].n, d_probs, S.pool.as<int32_t>(), S.work.as<double>(),
                       fac[i].work_off, fac[i].slot, S.err.as<int32_t>(), err_base + i, rst);
    }
    for (int i = 0; i < np; ++i) {
      if (fac[i].n < kWideRootMinN) continue;
      ProfScope ps_(RS_K_FACTOR, rst);
      launch_root_wide(cplx, d_fac + i, fac[i].n, d_probs, S.pool.as<int32_t>(),
                       S.work.as<double>(), fac[i].work_off, fac[i].slot, S.err.as<int32_t>(),
                       err_base + i, rst);
    }
    RS_HIP_CHECK(hipEventRecord(step_t[max_depth].b, rst));
    RS_HIP_CHECK(hipEventRecord(S.ev_root_done, rst));
    for (int p = 0; p < np; ++p) {
      ProbState &P = ps[p];
      const std::vector<int32_t> &J = P.J[0];
      const int n = (int)J.size();
      int32_t *d_idx = P.h->arena.alloc_n<int32_t>(std::max(n, 1));
      if (n)
        RS_HIP_CHECK(hipMemcpyAsync(d_idx, J.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, st));
      SweepBox sb;
      sb.k = 0;
      sb.r = n;
      sb.idx = d_idx;
      sb.T = sb.E = sb.F = nullptr;
      sb.G = fac[p].slot;
      rs_factor_s *h = P.h;
      h->root.depth = 0;
      h->root.boxes = {0};
      h->root.sweep = {sb};
      h->root.max_n = n;
      h->stats.root_size = n;
      h->stats.factor_doubles += (int64_t)n * n * es;
    }
  }
  // ---- upload the sweep descriptors
  for (int p = 0; p < np; ++p) {
    rs_factor_s *h = handles[p].get();
    for (LevelRec &lv : h->levels) {
      if (lv.d_sweep) continue;                 // uploaded when its step completed
      lv.partition_classes(mfma_max_n(cplx));
      lv.d_sweep = h->arena.alloc_n<SweepBox>((int64_t)lv.sweep.size());
      RS_HIP_CHECK(hipMemcpyAsync(lv.d_sweep, lv.sweep.data(), lv.sweep.size() * sizeof(SweepBox),
                                  hipMemcpyHostToDevice, st));
    }
    h->root.partition_classes(mfma_max_n(cplx));
    h->root.d_sweep = h->arena.alloc_n<SweepBox>(1);
    RS_HIP_CHECK(hipMemcpyAsync(h->root.d_sweep, h->root.sweep.data(), sizeof(SweepBox),
                                hipMemcpyHostToDevice, st));
  }
  // work of the caller's that may overlap the roots (it waits for them itself), then the
  // roots joined, the error index read back and checked
  if (hooks && np == 1 && hooks->after_roots)
    hooks->after_roots(handles[0].get(), st, S.ev_root_done);
  RS_HIP_CHECK(hipStreamWaitEvent(st, S.ev_root_done, 0));
  {
    auto tw = Clock::now();
    check_err(S.err, st, all_items, "factorization");
    wait_ms += ms_since(tw);
  }
  keep_alive.clear();
  RS_HIP_CHECK(hipStreamSynchronize(st));
  S.stage_reset();
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  // per-level device times: step s held depth maxdepth - s of each problem; the root last
  for (int p = 0; p < np; ++p) {
    rs_factor_s *h = handles[p].get();
    for (int step = 0; step < max_depth; ++step) {
      const int d = ps[p].t->maxdepth - step;
      if (d < 1 || !step_t[step].a) continue;
      float el = 0.f;
      RS_HIP_CHECK(hipEventElapsedTime(&el, step_t[step].a, step_t[step].b));
      rs_level_stats &e = level_entry(h, d);
      e.device_ms = el;
      e.plan_ms = step_t[step].plan_ms;
    }
    rs_level_stats &r = level_entry(h, 0);
    r.boxes = 1;
    r.n_total = r.max_n = (int32_t)h->stats.root_size;
    r.factor_doubles = (int64_t)h->stats.root_size * h->stats.root_size * es;
    if (step_t[max_depth].a) {
      float el = 0.f;
      RS_HIP_CHECK(hipEventElapsedTime(&el, step_t[max_depth].a, step_t[max_depth].b));
      r.device_ms = el;
    }
    std::stable_sort(h->level_stats.begin(), h->level_stats.end(),
                     [](const rs_level_stats &x, const rs_level_stats &y) {
                       return (x.depth == 0 ? -1 : x.depth) > (y.depth == 0 ? -1 : y.depth);
                     });
  }
  out.resize(np);
  for (int p = 0; p < np; ++p) {
    rs_factor_s *h = handles[p].get();
    h->box_J = std::move(ps[p].J);          // per-box active sets and skeletons (queries)
    h->box_skel = std::move(ps[p].skel);
    const Tree &tr = *ps[p].t;
    h->tree_first_child.assign(tr.first_child.begin(), tr.first_child.end());
    h->tree_nchild.assign(tr.nchild.begin(), tr.nchild.end());
    h->tree_begin = tr.begin;
    h->stats.n = h->n;
    h->stats.nbox = ps[p].t->nbox();
    h->stats.maxdepth = ps[p].t->maxdepth;
    h->stats.dim = h->dim;
    h->stats.complex_values = h->cplx ? 1 : 0;
    h->stats.factor_ms = ms;
    h->stats.plan_ms = plan_ms;
    h->stats.wait_ms = wait_ms;
    out[p] = handles[p].release();
  }
  // the per-box candidate lists and other planner state go to the background thread
  auto *left = new std::vector<ProbState>(std::move(ps));
  Reaper::get().defer([left] { delete left; });
}

}  // namespace

void factor_many(const std::vector<FactorRequest> &reqs, int launch_mode, hipStream_t st,
                 std::vector<rs_factor_s *> &out, const FactorHooks *hooks) {
  std::lock_guard<std::mutex> lock(g_factor_mutex);
  // Launches are typed by the scalar: real and complex problems are factored in two
  // groups (each problem's arithmetic is the same either way).
  std::vector<int> idx[2];
  for (int i = 0; i < (int)reqs.size(); ++i)
    idx[(reqs[i].k->kind == RS_HELM2D_CFIE || reqs[i].k->kind == RS_HELM3D_SL) ? 1 : 0]
        .push_back(i);
  if (idx[0].empty() || idx[1].empty()) {
    factor_group(reqs, launch_mode, st, out, hooks);
    return;
  }
  out.assign(reqs.size(), nullptr);
  try {
    for (int g = 0; g < 2; ++g) {
      std::vector<FactorRequest> sub;
      for (int i : idx[g]) sub.push_back(reqs[i]);
      std::vector<rs_factor_s *> o;
      factor_group(sub, launch_mode, st, o, nullptr);
      for (size_t j = 0; j < o.size(); ++j) out[idx[g][j]] = o[j];
    }
  } catch (...) {
    for (rs_factor_s *h : out) delete h;
    out.clear();
    throw;
  }
}

namespace {
// Wide-class scratch of one level at nrhs columns: every wide box at once when that fits
// kWideScratchCap doubles, else chunks of boxes (at least one box).
constexpr int64_t kWideScratchCap = int64_t(64) << 20;
int64_t wide_scratch_for(const LevelRec &lv, int nrhs, bool cplx) {
  const int cnt = (int)lv.sweep.size() - lv.n_small;
  if (cnt <= 0 || nrhs <= 0) return 0;
  const int64_t per = wide_scratch_doubles(1, lv.max_n_large, lv.max_r_large, nrhs, cplx);
  return std::min<int64_t>(per * cnt, std::max<int64_t>(per, kWideScratchCap));
}
int64_t wide_scratch_for(const rs_factor_s *h, int nrhs) {
  int64_t m = wide_scratch_for(h->root, nrhs, h->cplx);
  for (const LevelRec &lv : h->levels) m = std::max(m, wide_scratch_for(lv, nrhs, h->cplx));
  return m;
}
}  // namespace

namespace {
MvBox mv_box(const rs_factor_s *h, int b, const SweepBox &sb, int64_t save_off) {
  MvBox m{};
  m.k = sb.k;
  m.r = sb.r;
  m.idx = sb.idx;
  m.T = sb.T;
  m.save_off = save_off;
  m.prob = 0;
  m.nchild = h->tree_nchild[b];
  m.leaf = m.nchild == 0 ? 1 : 0;
  if (m.nchild > 8) throw std::runtime_error("matvec: a box has more than 8 children");
  for (int c = 0; c < m.nchild; ++c) m.child_begin[c] = h->tree_begin[h->tree_first_child[b] + c];
  return m;
}

MvLevel mv_upload(rs_factor_s *h, const std::vector<MvBox> &v, hipStream_t st) {
  MvLevel L;
  L.count = (int)v.size();
  for (const MvBox &m : v) {
    L.max_k = std::max(L.max_k, (int)m.k);
    L.max_r = std::max(L.max_r, (int)m.r);
    L.max_n = std::max(L.max_n, (int)(m.k + m.r));
  }
  if (!v.empty()) {
    L.d = h->arena.alloc_n<MvBox>((int64_t)v.size());
    RS_HIP_CHECK(hipMemcpyAsync(L.d, v.data(), v.size() * sizeof(MvBox), hipMemcpyHostToDevice, st));
  }
  return L;
}

// Builds the handle's forward-operator descriptors once (thread-safe).
MvPlan &mv_plan(rs_factor_s *h, hipStream_t st) {
  std::lock_guard<std::mutex> lock(h->mv_mu);
  if (h->mv) return *h->mv;
  auto plan = std::make_unique<MvPlan>();
  int64_t save = 0;
  for (const LevelRec &lv : h->levels) {
    std::vector<MvBox> v;
    for (size_t i = 0; i < lv.sweep.size(); ++i) {
      v.push_back(mv_box(h, lv.boxes[i], lv.sweep[i], save));
      save += lv.sweep[i].k;
    }
    plan->levels.push_back(mv_upload(h, v, st));
  }
  plan->root = mv_upload(h, {mv_box(h, 0, h->root.sweep[0], 0)}, st);
  plan->save_rows = save;
  plan->d_prob = h->arena.alloc_n<ProbDev>(1);
  RS_HIP_CHECK(hipMemcpyAsync(plan->d_prob, &h->prob, sizeof(ProbDev), hipMemcpyHostToDevice, st));
  RS_HIP_CHECK(hipStreamSynchronize(st));     // host descriptor arrays go out of scope
  h->mv = std::move(plan);
  return *h->mv;
}
}  // namespace

void matvec_one(rs_factor_s *h, const void *X, int64_t ldx, void *Y, int64_t ldy, int nrhs,
                hipStream_t st) {
  if (nrhs == 0) return;
  const MvPlan &P = mv_plan(h, st);
  const int64_t n = h->n;
  const bool cplx = h->cplx;
  const size_t es = cplx ? 2 : 1;
  const size_t cols = (size_t)nrhs * es * sizeof(double);
  double *W = nullptr, *Yw = nullptr, *save = nullptr;
  RS_HIP_CHECK(hipMallocAsync((void **)&W, (size_t)n * cols, st));
  struct Freer {
    double *p;
    hipStream_t st;
    ~Freer() {
      if (p) (void)hipFreeAsync(p, st);
    }
  } f1{W, st};
  RS_HIP_CHECK(hipMallocAsync((void **)&Yw, (size_t)n * cols, st));
  Freer f2{Yw, st};
  RS_HIP_CHECK(hipMallocAsync((void **)&save, std::max<size_t>((size_t)P.save_rows * cols, 8), st));
  Freer f3{save, st};
  launch_permute_in(cplx, static_cast<const double *>(X), ldx, W, h->d_perm, n, nrhs, st);
  RS_HIP_CHECK(hipMemsetAsync(Yw, 0, (size_t)n * cols, st));
  for (const MvLevel &L : P.levels)
    launch_mv_up(cplx, L.d, L.count, L.max_k, W, nrhs, save, st);
  launch_mv_diag(cplx, P.root.d, P.root.count, P.root.max_n, P.d_prob, W, save, Yw, nrhs, st);
  for (auto it = P.levels.rbegin(); it != P.levels.rend(); ++it) {
    launch_mv_lift(cplx, it->d, it->count, it->max_r, Yw, nrhs, st);
    launch_mv_diag(cplx, it->d, it->count, it->max_n, P.d_prob, W, save, Yw, nrhs, st);
  }
  launch_permute_out(cplx, static_cast<double *>(Y), ldy, Yw, h->d_perm, n, nrhs, st);
}

bool is_device_buffer(const void *p, size_t bytes) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();       // unknown to the runtime: plain host memory
    return false;
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged) return false;
  int cur = 0;
  RS_HIP_CHECK(hipGetDevice(&cur));
  if (a.device != cur)
    throw UserError{RS_EINVAL, "buffer is on device " + std::to_string(a.device) +
                                   ", the current device is " + std::to_string(cur)};
  void *base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) == hipSuccess && base) {
    if (static_cast<const char *>(p) + bytes > static_cast<const char *>(base) + size)
      throw UserError{RS_EINVAL, "buffer runs past the end of its device allocation"};
  } else {
    (void)hipGetLastError();
  }
  return true;
}

std::shared_ptr<SharedEvent> record_completion(hipStream_t st) {
  auto e = std::make_shared<SharedEvent>();
  RS_HIP_CHECK(hipEventCreateWithFlags(&e->ev, hipEventDisableTiming));
  RS_HIP_CHECK(hipEventRecord(e->ev, st));
  return e;
}

void note_inflight(rs_factor_s *h, const std::shared_ptr<SharedEvent> &e) {
  std::lock_guard<std::mutex> lock(h->inflight_mu);
  // drop completed events (a stalled one on another stream only delays the pruning)
  size_t keep = 0;
  for (auto &x : h->inflight)
    if (hipEventQuery(x->ev) == hipErrorNotReady) h->inflight[keep++] = x;
  h->inflight.resize(keep);
  h->inflight.push_back(e);
}

void note_inflight(rs_factor_s *h, hipStream_t st) { note_inflight(h, record_completion(st)); }

bool has_inflight(rs_factor_s *h) {
  std::lock_guard<std::mutex> lock(h->inflight_mu);
  size_t keep = 0;
  for (auto &x : h->inflight)
    if (hipEventQuery(x->ev) == hipErrorNotReady) h->inflight[keep++] = x;
  h->inflight.resize(keep);
  return keep > 0;
}

void solve_one(rs_factor_s *h, void *Bv, int64_t ldb, int nrhs, int launch_mode,
               hipStream_t st, hipEvent_t roots_ready) {
  if (nrhs == 0) return;
  const int es = h->cplx ? 2 : 1;
  double *W = nullptr;
  RS_HIP_CHECK(hipMallocAsync((void **)&W, (size_t)h->n * nrhs * sizeof(double) * es, st));
  struct Freer {
    double *W;
    hipStream_t st;
    ~Freer() {
      if (W) (void)hipFreeAsync(W, st);
    }
  } freer{W, st};
  const int64_t wide_sz = wide_scratch_for(h, nrhs);
  double *wide = nullptr;
  if (wide_sz > 0)
    RS_HIP_CHECK(hipMallocAsync((void **)&wide, (size_t)wide_sz * sizeof(double), st));
  Freer wide_freer{wide, st};
  solve_one_into(h, Bv, ldb, nrhs, launch_mode, st, W, wide, wide_sz, roots_ready);
}

int64_t solve_wide_min_doubles(const rs_factor_s *h, int nrhs) {
  int64_t m = 0;
  auto one = [&](const LevelRec &lv) {
    if ((int)lv.sweep.size() > lv.n_small && lv.max_r_large > 0)
      m = std::max(m, wide_scratch_doubles(1, lv.max_n_large, lv.max_r_large, nrhs, h->cplx));
  };
  one(h->root);
  for (const LevelRec &lv : h->levels) one(lv);
  return m;
}

int64_t solve_wide_doubles(const rs_factor_s *h, int nrhs) { return wide_scratch_for(h, nrhs); }

// One level's sweep of a solve (upward or downward), as every solve issues it: the MFMA
// class in one launch (or one per box), then the wide class.
void sweep_level(const rs_factor_s *h, const LevelRec &lv, bool up, double *W, int nrhs,
                 bool per_box, double *wide, int64_t wide_sz, hipStream_t st) {
  const bool cplx = h->cplx;
  const int cnt = (int)lv.sweep.size();
  const int fam = up ? RS_K_SWEEP_UP : RS_K_SWEEP_DOWN;
  if (prof_on()) {
    Work w;
    for (const SweepBox &sb : lv.sweep)
      w += up ? work_sweep_up(sb.k, sb.r, nrhs, cplx) : work_sweep_down(sb.k, sb.r, nrhs, cplx);
    prof_add_work(fam, w);
  }
  if (per_box) {
    for (int i = 0; i < cnt; ++i) {
      ProfScope ps_(fam, st);
      const int n = lv.sweep[i].k + lv.sweep[i].r;
      if (i < lv.n_small)
        launch_sweep_mfma(cplx, up, lv.d_sweep, i, 1, W, nrhs, n, st);
      else
        launch_wide_level(cplx, up, lv.d_sweep + i, 1, n, lv.sweep[i].k, lv.sweep[i].r, W,
                          nrhs, wide, wide_sz, st);
    }
  } else {
    ProfScope ps_(fam, st);
    launch_sweep_mfma(cplx, up, lv.d_sweep, 0, lv.n_small, W, nrhs, lv.max_n_small, st);
    launch_wide_level(cplx, up, lv.d_sweep + lv.n_small, cnt - lv.n_small, lv.max_n_large,
                      lv.max_k_large, lv.max_r_large, W, nrhs, wide, wide_sz, st);
  }
}

void permute_rhs(const rs_factor_s *h, bool in, void *Bv, int64_t ldb, double *W, int nrhs,
                 hipStream_t st) {
  Work wperm;
  wperm.bytes = 16.0 * (h->cplx ? 2 : 1) * h->n * nrhs + 8.0 * h->n;
  prof_add_work(RS_K_PERMUTE, wperm);
  ProfScope ps_(RS_K_PERMUTE, st);
  double *B = static_cast<double *>(Bv);
  if (in) launch_permute_in(h->cplx, B, ldb, W, h->d_perm, h->n, nrhs, st);
  else launch_permute_out(h->cplx, B, ldb, W, h->d_perm, h->n, nrhs, st);
}

rs_factor_s *factor_and_solve(const FactorRequest &req, int launch_mode, hipStream_t st,
                              void *B, int64_t ldb, int nrhs) {
  const bool per_box = launch_mode == RS_LAUNCH_PER_BOX;
  struct Run {
    double *W = nullptr, *wide = nullptr;
    int64_t wide_sz = 0;
    hipStream_t side = nullptr;
    hipEvent_t ups = nullptr;
    ~Run() {
      if (ups) (void)hipEventDestroy(ups);
    }
    // wide-class staging of at least need doubles, stream-ordered on s
    void ensure_wide(int64_t need, hipStream_t s) {
      if (need <= wide_sz) return;
      if (wide) RS_HIP_CHECK(hipFreeAsync(wide, s));
      wide = nullptr;
      RS_HIP_CHECK(hipMallocAsync((void **)&wide, (size_t)need * sizeof(double), s));
      wide_sz = need;
    }
  } run;
  FactorHooks hk;
  hk.begin = [&](rs_factor_s *h, hipStream_t side) {
    run.side = side;
    const size_t es = h->cplx ? 2 : 1;
    RS_HIP_CHECK(hipMallocAsync((void **)&run.W, (size_t)h->n * nrhs * sizeof(double) * es, side));
    permute_rhs(h, true, B, ldb, run.W, nrhs, side);
  };
  hk.level = [&](rs_factor_s *h, const LevelRec &lv, hipStream_t side) {
    run.ensure_wide(wide_scratch_for(lv, nrhs, h->cplx), side);
    sweep_level(h, lv, true, run.W, nrhs, per_box, run.wide, run.wide_sz, side);
  };
  hk.after_roots = [&](rs_factor_s *h, hipStream_t s, hipEvent_t roots) {
    // the upward sweeps queued on the side stream, then the roots
    RS_HIP_CHECK(hipEventCreateWithFlags(&run.ups, hipEventDisableTiming));
    RS_HIP_CHECK(hipEventRecord(run.ups, run.side));
    RS_HIP_CHECK(hipStreamWaitEvent(s, run.ups, 0));
    RS_HIP_CHECK(hipStreamWaitEvent(s, roots, 0));
    run.ensure_wide(wide_scratch_for(h, nrhs), s);
    sweep_level(h, h->root, true, run.W, nrhs, per_box, run.wide, run.wide_sz, s);
    for (auto it = h->levels.rbegin(); it != h->levels.rend(); ++it)
      sweep_level(h, *it, false, run.W, nrhs, per_box, run.wide, run.wide_sz, s);
    permute_rhs(h, false, B, ldb, run.W, nrhs, s);
  };
  std::vector<FactorRequest> reqs{req};
  std::vector<rs_factor_s *> hs;
  // the solve's buffers, released behind its work on st (also on errors: the factor call
  // drains its own streams before it returns or throws)
  struct Freer {
    Run &r;
    hipStream_t st;
    ~Freer() {
      if (r.W) (void)hipFreeAsync(r.W, st);
      if (r.wide) (void)hipFreeAsync(r.wide, st);
    }
  } freer{run, st};
  factor_many(reqs, launch_mode, st, hs, nrhs > 0 ? &hk : nullptr);
  return hs[0];
}

void solve_one_into(rs_factor_s *h, void *Bv, int64_t ldb, int nrhs, int launch_mode,
                    hipStream_t st, double *W, double *wide, int64_t wide_sz,
                    hipEvent_t roots_ready) {
  if (nrhs == 0) return;
  const bool per_box = launch_mode == RS_LAUNCH_PER_BOX;
  permute_rhs(h, true, Bv, ldb, W, nrhs, st);
  for (const LevelRec &lv : h->levels) sweep_level(h, lv, true, W, nrhs, per_box, wide, wide_sz, st);
  if (roots_ready) RS_HIP_CHECK(hipStreamWaitEvent(st, roots_ready, 0));
  sweep_level(h, h->root, true, W, nrhs, per_box, wide, wide_sz, st);
  for (auto it = h->levels.rbegin(); it != h->levels.rend(); ++it)
    sweep_level(h, *it, false, W, nrhs, per_box, wide, wide_sz, st);
  permute_rhs(h, false, Bv, ldb, W, nrhs, st);
}

}  // namespace rs

namespace rs {

namespace {
struct LaunchRec {
  int64_t seg_off;
  int nseg, nblocks, max_nrhs, max_n;
  bool up, mfma;
  int64_t wide_off;   // wide class (mfma false): T.wide[wide_off, wide_off + nwide)
  int nwide;
};
// Wide-class boxes of one handle's level (launch_wide_level arguments).
struct WideRec {
  const SweepBox *boxes;
  double *W;
  int count, max_n, max_k, max_r, nrhs;
};
void release_host_vector(void *p) { delete static_cast<std::vector<char> *>(p); }
}  // namespace

namespace {

// Launch tables of one group's solve (requests whose handles share one scalar type):
// permutation segments, then upward steps (finest level first), the roots, then
// downward steps; each launch's segments are contiguous.  W is the group's workspace.
struct SolveTables {
  bool cplx = false;
  int nq = 0;
  int64_t max_elems = 0;
  int max_nrhs = 0;
  std::vector<PermSeg> perm;
  std::vector<SweepSeg> segs;
  std::vector<WideRec> wide;
  int64_t wide_scratch = 0;          // doubles
  std::vector<LaunchRec> launches;
};

int64_t group_workspace(const std::vector<SolveRequest> &rq) {
  int64_t wtot = 0;
  for (const SolveRequest &q : rq) wtot += q.h->n * (int64_t)q.nrhs;
  return wtot * (rq.empty() || !rq[0].h->cplx ? 1 : 2);    // doubles
}

SolveTables build_tables(const std::vector<SolveRequest> &rq, double *W) {
  SolveTables T;
  const int nq = (int)rq.size();
  T.nq = nq;
  T.cplx = rq[0].h->cplx;
  const int es = T.cplx ? 2 : 1;
  std::vector<int64_t> woff(nq);
  int64_t wtot = 0;
  int max_levels = 0;
  for (int i = 0; i < nq; ++i) {
    woff[i] = wtot;
    wtot += rq[i].h->n * (int64_t)rq[i].nrhs;
    max_levels = std::max(max_levels, (int)rq[i].h->levels.size());
  }
  T.perm.resize(nq);
  for (int i = 0; i < nq; ++i) {
    PermSeg &p = T.perm[i];
    p.B = static_cast<double *>(rq[i].B);
    p.ldb = rq[i].ldb;
    p.W = W + woff[i] * es;
    p.perm = rq[i].h->d_perm;
    p.n = rq[i].h->n;
    p.nrhs = rq[i].nrhs;
    p.pad = 0;
    T.max_elems = std::max<int64_t>(T.max_elems, rq[i].h->n * (int64_t)rq[i].nrhs);
    T.max_nrhs = std::max(T.max_nrhs, rq[i].nrhs);
  }
  auto add_step = [&](bool up, auto level_of) {
    for (int mfma = 1; mfma >= 0; --mfma) {
      LaunchRec L{(int64_t)T.segs.size(), 0, 0, 0, 0, up, mfma == 1, (int64_t)T.wide.size(), 0};
      for (int i = 0; i < nq; ++i) {
        const LevelRec *lv = level_of(rq[i].h);
        if (!lv || lv->sweep.empty()) continue;
        const int lo = mfma ? 0 : lv->n_small;
        const int cnt = mfma ? lv->n_small : (int)lv->sweep.size() - lv->n_small;
        if (cnt <= 0) continue;
        if (!mfma) {
          T.wide.push_back(WideRec{lv->d_sweep + lo, W + woff[i] * es, cnt, lv->max_n_large,
                                   lv->max_k_large, lv->max_r_large, rq[i].nrhs});
          T.wide_scratch = std::max(T.wide_scratch, wide_scratch_for(*lv, rq[i].nrhs, T.cplx));
          L.nwide++;
          continue;
        }
        SweepSeg s;
        s.boxes = lv->d_sweep + lo;
        s.W = W + woff[i] * es;
        s.count = cnt;
        s.nrhs = rq[i].nrhs;
        s.block0 = L.nblocks;
        s.pad = 0;
        T.segs.push_back(s);
        L.nseg++;
        L.nblocks += s.count;
        L.max_nrhs = std::max(L.max_nrhs, s.nrhs);
        L.max_n = std::max(L.max_n, mfma ? lv->max_n_small : lv->max_n_large);
      }
      if (L.nseg || L.nwide) T.launches.push_back(L);
    }
  };
  for (int t = 0; t < max_levels; ++t)
    add_step(true, [t](rs_factor_s *h) -> const LevelRec * {
      return t < (int)h->levels.size() ? &h->levels[t] : nullptr;
    });
  add_step(true, [](rs_factor_s *h) -> const LevelRec * { return &h->root; });
  for (int t = max_levels - 1; t >= 0; --t)
    add_step(false, [t](rs_factor_s *h) -> const LevelRec * {
      return t < (int)h->levels.size() ? &h->levels[t] : nullptr;
    });
  return T;
}

// Packs the tables (PermSeg array, then SweepSeg array) into one host buffer.
std::vector<char> *pack_tables(const SolveTables &T) {
  const size_t perm_bytes = T.perm.size() * sizeof(PermSeg);
  const size_t seg_bytes = T.segs.size() * sizeof(SweepSeg);
  auto *host = new std::vector<char>(perm_bytes + seg_bytes);
  std::memcpy(host->data(), T.perm.data(), perm_bytes);
  if (seg_bytes) std::memcpy(host->data() + perm_bytes, T.segs.data(), seg_bytes);
  return host;
}

// The kernel launches of a group's solve; kernels only (no copies or fills), so the
// sequence can be captured into a graph.
void enqueue_group(const SolveTables &T, const char *dtab, double *wide, hipStream_t st) {
  const PermSeg *d_perm = reinterpret_cast<const PermSeg *>(dtab);
  const SweepSeg *d_segs =
      reinterpret_cast<const SweepSeg *>(dtab + T.perm.size() * sizeof(PermSeg));
  {
    ProfScope ps_(RS_K_PERMUTE, st);
    launch_permute_seg(T.cplx, d_perm, T.nq, T.max_elems, T.max_nrhs, true, st);
  }
  for (const LaunchRec &L : T.launches) {
    ProfScope ps_(L.up ? RS_K_SWEEP_UP : RS_K_SWEEP_DOWN, st);
    if (L.nseg)
      launch_sweep_seg(T.cplx, L.up, d_segs + L.seg_off, L.nseg, L.nblocks, L.max_nrhs, L.max_n,
                       st);
    for (int w = 0; w < L.nwide; ++w) {
      const WideRec &R = T.wide[L.wide_off + w];
      launch_wide_level(T.cplx, L.up, R.boxes, R.count, R.max_n, R.max_k, R.max_r, R.W, R.nrhs,
                        wide, T.wide_scratch, st);
    }
  }
  {
    ProfScope ps_(RS_K_PERMUTE, st);
    launch_permute_seg(T.cplx, d_perm, T.nq, T.max_elems, T.max_nrhs, false, st);
  }
}

void solve_group(const std::vector<SolveRequest> &rq, hipStream_t st) {
  if (rq.empty()) return;
  double *W = nullptr;
  RS_HIP_CHECK(hipMallocAsync((void **)&W, (size_t)group_workspace(rq) * sizeof(double), st));
  const SolveTables T = build_tables(rq, W);
  // one upload of all tables; the host copy is released by a stream callback
  std::vector<char> *host = pack_tables(T);
  char *dtab = nullptr;
  RS_HIP_CHECK(hipMallocAsync((void **)&dtab, host->size(), st));
  RS_HIP_CHECK(hipMemcpyAsync(dtab, host->data(), host->size(), hipMemcpyHostToDevice, st));
  RS_HIP_CHECK(hipLaunchHostFunc(st, release_host_vector, host));
  double *wide = nullptr;
  if (T.wide_scratch > 0)
    RS_HIP_CHECK(hipMallocAsync((void **)&wide, (size_t)T.wide_scratch * sizeof(double), st));
  enqueue_group(T, dtab, wide, st);
  if (wide) RS_HIP_CHECK(hipFreeAsync(wide, st));
  RS_HIP_CHECK(hipFreeAsync(dtab, st));
  RS_HIP_CHECK(hipFreeAsync(W, st));
}

}  // namespace

void solve_many(const std::vector<SolveRequest> &reqs, hipStream_t st) {
  std::vector<SolveRequest> rq[2];
  for (const SolveRequest &q : reqs)
    if (q.nrhs > 0) rq[q.h->cplx ? 1 : 0].push_back(q);
  solve_group(rq[0], st);
  solve_group(rq[1], st);
}

// ---- captured solves
SolvePlan::~SolvePlan() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  for (rs_factor_s *h : handles) h->busy.fetch_sub(1);
}

SolvePlan *make_plan(const std::vector<SolveRequest> &reqs) {
  std::unique_ptr<SolvePlan> plan(new SolvePlan());
  std::vector<SolveRequest> rq[2];
  for (const SolveRequest &q : reqs) {
    plan->handles.push_back(q.h);
    q.h->busy.fetch_add(1);
    if (q.nrhs > 0) rq[q.h->cplx ? 1 : 0].push_back(q);
  }
  // persistent workspace and tables, uploaded before capture
  std::vector<SolveTables> tabs;
  std::vector<char *> dtabs;
  std::vector<double *> wides;
  for (int g = 0; g < 2; ++g) {
    if (rq[g].empty()) continue;
    void *W = nullptr;
    RS_HIP_CHECK(hipMalloc(&W, std::max<size_t>((size_t)group_workspace(rq[g]), 1) * sizeof(double)));
    plan->bufs.push_back(W);
    tabs.push_back(build_tables(rq[g], static_cast<double *>(W)));
    std::unique_ptr<std::vector<char>> host(pack_tables(tabs.back()));
    void *dtab = nullptr;
    RS_HIP_CHECK(hipMalloc(&dtab, std::max<size_t>(host->size(), 1)));
    plan->bufs.push_back(dtab);
    RS_HIP_CHECK(hipMemcpy(dtab, host->data(), host->size(), hipMemcpyHostToDevice));
    dtabs.push_back(static_cast<char *>(dtab));
    void *wide = nullptr;
    if (tabs.back().wide_scratch > 0) {
      RS_HIP_CHECK(hipMalloc(&wide, (size_t)tabs.back().wide_scratch * sizeof(double)));
      plan->bufs.push_back(wide);
    }
    wides.push_back(static_cast<double *>(wide));
  }
  hipStream_t cs = nullptr;
  RS_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } guard{cs};
  {
    CaptureScope capture;              // the profiler records no events while capturing
    RS_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
      for (size_t g = 0; g < tabs.size(); ++g) enqueue_group(tabs[g], dtabs[g], wides[g], cs);
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(cs, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    RS_HIP_CHECK(hipStreamEndCapture(cs, &plan->graph));
  }
  RS_HIP_CHECK(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
  return plan.release();
}

void launch_plan(SolvePlan *p, hipStream_t st) { RS_HIP_CHECK(hipGraphLaunch(p->exec, st)); }

}  // namespace rs
