// C ABI entry points: argument validation, error translation, object lifetime.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "runtime.h"
#include "pool.h"

namespace rs {

thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

template <class F>
rs_status guarded(F &&f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const UserError &e) {
    g_last_error = e.what;
    return e.code;
  } catch (const DeviceError &e) {
    g_last_error = e.what;
    return RS_EDEVICE;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return RS_ENOMEM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return RS_EDEVICE;
  } catch (...) {
    g_last_error = "unknown error";
    return RS_EDEVICE;
  }
}

[[noreturn]] void fail(rs_status code, const std::string &msg) { throw UserError{code, msg}; }

bool all_finite(const double *p, int64_t n) {
  // branch-free over blocks (the compiler vectorizes the inner loop), early out per block
  constexpr int64_t kBlock = 4096;
  for (int64_t i0 = 0; i0 < n; i0 += kBlock) {
    const int64_t i1 = std::min(n, i0 + kBlock);
    bool ok = true;
    for (int64_t i = i0; i < i1; ++i) ok &= std::isfinite(p[i]);
    if (!ok) return false;
  }
  return true;
}

void validate_kernel(const rs_kernel *k, const Tree &t, const double *points,
                     const double *weights, double eps) {
  if (!k || !points || !weights) fail(RS_EINVAL, "NULL kernel, points or weights");
  if (k->kind != RS_LAP2D_SL && k->kind != RS_LAP2D_DL && k->kind != RS_LAP3D_SL &&
      k->kind != RS_HELM2D_CFIE && k->kind != RS_HELM3D_SL)
    fail(RS_EINVAL, "unknown kernel kind");
  const int want_dim = (k->kind == RS_LAP3D_SL || k->kind == RS_HELM3D_SL) ? 3 : 2;
  if (k->dim != want_dim || t.dim != want_dim) fail(RS_EINVAL, "kernel dimension mismatch");
  if ((k->kind == RS_LAP2D_DL || k->kind == RS_HELM2D_CFIE) && (!k->normals || !k->curvature))
    fail(RS_EINVAL, "double-layer kernel needs normals and curvature");
  if (k->kind == RS_HELM2D_CFIE &&
      (!(k->wavenumber > 0.0) || !std::isfinite(k->wavenumber) || !std::isfinite(k->eta)))
    fail(RS_EINVAL, "Helmholtz kernel needs a finite wavenumber > 0 and a finite eta");
  if (k->kind == RS_HELM3D_SL && (!(k->wavenumber > 0.0) || !std::isfinite(k->wavenumber)))
    fail(RS_EINVAL, "Helmholtz kernel needs a finite wavenumber > 0");
  if (k->proxy_points < 8 || k->proxy_points > 4096) fail(RS_EINVAL, "proxy_points out of range");
  if (k->id_mode != RS_ID_CPQR && k->id_mode != RS_ID_SKETCH) fail(RS_EINVAL, "unknown id_mode");
  if (k->id_mode == RS_ID_SKETCH && (k->oversample < 0 || k->oversample > 4096))
    fail(RS_EINVAL, "oversample out of range");
  if (!(k->proxy_ratio > 0.5 * std::sqrt((double)want_dim)) || !(k->proxy_ratio < 16.0))
    fail(RS_EINVAL, "proxy_ratio must exceed half the box diagonal");
  if (!std::isfinite(k->identity)) fail(RS_EINVAL, "non-finite identity coefficient");
  if (!(eps >= 0.0) || !std::isfinite(eps)) fail(RS_EINVAL, "eps must be finite and >= 0");
  // per-point checks, blocks of points on the host pool; each check that fails anywhere
  // sets its bit, and the first failed check in the order below is reported
  const int64_t n = t.n;
  const int dim = t.dim;
  constexpr int64_t kBlk = 8192;
  std::atomic<int> bad{0};
  parallel_for((int)((n + kBlk - 1) / kBlk), [&](int blk) {
    const int64_t i0 = blk * kBlk, i1 = std::min(n, i0 + kBlk), m = i1 - i0;
    int f = 0;
    if (!all_finite(points + i0 * dim, m * dim) || !all_finite(weights + i0, m)) f |= 1;
    bool pos = true;
    for (int64_t i = i0; i < i1; ++i) pos &= weights[i] > 0.0;
    if (!pos) f |= 2;
    if (k->normals && !all_finite(k->normals + i0 * dim, m * dim)) f |= 4;
    if (k->curvature && !all_finite(k->curvature + i0, m)) f |= 8;
    // the points must be the ones the tree was built on
    bool same = true;
    for (int64_t i = i0; i < i1; ++i)
      for (int a = 0; a < dim; ++a)
        same &= points[t.perm[i] * dim + a] == t.coords[(size_t)a * n + i];
    if (!same) f |= 16;
    if (f) bad.fetch_or(f);
  }, 1);
  const int b = bad.load();
  if (b & 1) fail(RS_EINVAL, "non-finite points or weights");
  if (b & 2) fail(RS_EINVAL, "weights must be positive");
  if (b & 4) fail(RS_EINVAL, "non-finite normals");
  if (b & 8) fail(RS_EINVAL, "non-finite curvature");
  if (b & 16) fail(RS_EINVAL, "points differ from the tree's points");
}

hipStream_t stream_of(const rs_options *o) {
  return o ? static_cast<hipStream_t>(o->stream) : nullptr;
}

int mode_of(const rs_options *o) {
  if (!o) return RS_LAUNCH_LEVEL;
  if (o->launch_mode != RS_LAUNCH_LEVEL && o->launch_mode != RS_LAUNCH_PER_BOX)
    fail(RS_EINVAL, "unknown launch mode");
  return o->launch_mode;
}

// Bytes the device's default stream-ordered pool keeps after its buffers are freed.  The
// solves take their workspaces (the permuted right-hand sides, the wide class's staging:
// 268 MB for 512 columns at N = 65536) with hipMallocAsync and return them at the end;
// with the pool's default threshold of zero every call mapped and unmapped them again.
constexpr uint64_t kPoolKeepBytes = 4ull << 30;

void require_device() {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
    fail(RS_EDEVICE, "no HIP device available");
  // once per device: the default pool keeps up to kPoolKeepBytes of freed memory
  static std::mutex mu;
  static std::vector<char> done;
  int dev = 0;
  RS_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)done.size() <= dev) done.resize(dev + 1, 0);
  if (done[dev]) return;
  hipMemPool_t pool = nullptr;
  RS_HIP_CHECK(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t keep = kPoolKeepBytes;
  RS_HIP_CHECK(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  done[dev] = 1;
}

}  // namespace rs

using namespace rs;

extern "C" {

const char *rs_last_error(void) { return g_last_error.c_str(); }

int32_t rs_device_count(void) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return 0;
  return count;
}

rs_status rs_build_tree(int32_t dim, int64_t n, const double *points, int32_t leaf_size,
                        rs_tree *out) {
  return guarded([&]() -> rs_status {
    if (!out || !points) fail(RS_EINVAL, "NULL argument");
    if (dim != 2 && dim != 3) fail(RS_EINVAL, "dim must be 2 or 3");
    if (n < 1 || n > INT32_MAX - 1) fail(RS_EINVAL, "n out of range");
    if (leaf_size < 1) fail(RS_EINVAL, "leaf_size must be positive");
    if (!all_finite(points, n * dim)) fail(RS_EINVAL, "non-finite point coordinate");
    rs_tree t = new rs_tree_s();
    t->t.build(dim, n, points, leaf_size);
    *out = t;
    return RS_OK;
  });
}

rs_status rs_tree_info(rs_tree t, int64_t *nbox, int32_t *maxdepth) {
  return guarded([&]() -> rs_status {
    if (!t) fail(RS_EINVAL, "NULL tree");
    if (nbox) *nbox = t->t.nbox();
    if (maxdepth) *maxdepth = t->t.maxdepth;
    return RS_OK;
  });
}

rs_status rs_tree_export(rs_tree t, int64_t *perm, int32_t *depth, int32_t *parent,
                         int64_t *begin, int64_t *end, double *center, double *side) {
  return guarded([&]() -> rs_status {
    if (!t) fail(RS_EINVAL, "NULL tree");
    const Tree &T = t->t;
    const int nb = T.nbox();
    if (perm) std::memcpy(perm, T.perm.data(), T.n * sizeof(int64_t));
    for (int b = 0; b < nb; ++b) {
      if (depth) depth[b] = T.depth[b];
      if (parent) parent[b] = T.parent[b];
      if (begin) begin[b] = T.begin[b];
      if (end) end[b] = T.end[b];
      if (side) side[b] = T.side[b];
      if (center)
        for (int a = 0; a < T.dim; ++a) center[(int64_t)b * T.dim + a] = T.center[3 * b + a];
    }
    return RS_OK;
  });
}

void rs_tree_free(rs_tree t) { delete t; }

rs_status rs_factor_ex(const rs_kernel *k, rs_tree t, const double *points,
                       const double *weights, double eps, const rs_options *opts,
                       rs_handle *out) {
  return guarded([&]() -> rs_status {
    if (!out || !t) fail(RS_EINVAL, "NULL argument");
    validate_kernel(k, t->t, points, weights, eps);
    const int mode = mode_of(opts);
    require_device();
    std::vector<FactorRequest> reqs{{k, &t->t, points, weights, eps}};
    std::vector<rs_factor_s *> hs;
    factor_many(reqs, mode, stream_of(opts), hs);
    *out = hs[0];
    return RS_OK;
  });
}

rs_status rs_factor_solve_ex(const rs_kernel *k, rs_tree t, const double *points,
                             const double *weights, double eps, const rs_options *opts,
                             void *B, int64_t ldb, int32_t nrhs, rs_handle *out) {
  return guarded([&]() -> rs_status {
    if (!out || !t) fail(RS_EINVAL, "NULL argument");
    validate_kernel(k, t->t, points, weights, eps);
    if (nrhs < 0) fail(RS_EINVAL, "nrhs must be >= 0");
    const int64_t n = t->t.n;
    if (nrhs > 0 && !B) fail(RS_EINVAL, "NULL right-hand side");
    if (nrhs > 0 && ldb < n) fail(RS_EINVAL, "ldb < n");
    const bool cplx = k->kind == RS_HELM2D_CFIE || k->kind == RS_HELM3D_SL;
    const size_t es = cplx ? 16 : 8;
    if (nrhs > 0 && !is_device_buffer(B, ((size_t)(nrhs - 1) * (size_t)ldb + (size_t)n) * es))
      fail(RS_EINVAL, "rs_factor_solve_ex takes device right-hand sides only");
    const int mode = mode_of(opts);
    require_device();
    *out = factor_and_solve(FactorRequest{k, &t->t, points, weights, eps}, mode,
                            stream_of(opts), B, ldb, nrhs);
    return RS_OK;
  });
}

rs_status rs_factor(const rs_kernel *k, rs_tree t, const double *points, const double *weights,
                    double eps, rs_handle *out) {
  return rs_factor_ex(k, t, points, weights, eps, nullptr, out);
}

rs_status rs_factor_batched(int32_t count, const rs_kernel *kernels, const rs_tree *trees,
                            const double *const *points, const double *const *weights,
                            const double *eps, const rs_options *opts, rs_handle *out) {
  return guarded([&]() -> rs_status {
    if (count < 0) fail(RS_EINVAL, "count must be >= 0");
    if (count == 0) return RS_OK;
    if (!kernels || !trees || !points || !weights || !eps || !out) fail(RS_EINVAL, "NULL argument");
    std::vector<FactorRequest> reqs(count);
    for (int i = 0; i < count; ++i) {
      if (!trees[i]) fail(RS_EINVAL, "NULL tree");
      validate_kernel(&kernels[i], trees[i]->t, points[i], weights[i], eps[i]);
      reqs[i] = FactorRequest{&kernels[i], &trees[i]->t, points[i], weights[i], eps[i]};
    }
    const int mode = mode_of(opts);
    require_device();
    std::vector<rs_factor_s *> hs;
    factor_many(reqs, mode, stream_of(opts), hs);
    for (int i = 0; i < count; ++i) out[i] = hs[i];
    return RS_OK;
  });
}

rs_status rs_solve_batched(int32_t count, const rs_handle *h, void *const *B,
                           const int64_t *ldb, const int32_t *nrhs, const rs_options *opts) {
  return guarded([&]() -> rs_status {
    if (count < 0) fail(RS_EINVAL, "count must be >= 0");
    if (count == 0) return RS_OK;
    if (!h || !B || !ldb || !nrhs) fail(RS_EINVAL, "NULL argument");
    std::vector<SolveRequest> reqs(count);
    for (int i = 0; i < count; ++i) {
      if (!h[i]) fail(RS_EINVAL, "NULL handle");
      if (nrhs[i] < 0) fail(RS_EINVAL, "nrhs must be >= 0");
      if (nrhs[i] > 0 && !B[i]) fail(RS_EINVAL, "NULL right-hand side");
      if (ldb[i] < h[i]->n) fail(RS_EINVAL, "ldb < n");
      reqs[i] = SolveRequest{h[i], B[i], ldb[i], nrhs[i]};
    }
    if (opts && opts->launch_mode != RS_LAUNCH_LEVEL)
      fail(RS_EINVAL, "batched solves use per-level launches");
    for (int i = 0; i < count; ++i) h[i]->busy.fetch_add(1);
    struct Dec {
      const rs_handle *h;
      int n;
      ~Dec() {
        for (int i = 0; i < n; ++i) h[i]->busy.fetch_sub(1);
      }
    } dec{h, count};
    for (int i = 0; i < count; ++i) {
      if (nrhs[i] == 0) continue;
      const size_t es = h[i]->cplx ? 16 : 8;
      if (!is_device_buffer(B[i], ((size_t)(nrhs[i] - 1) * (size_t)ldb[i] + (size_t)h[i]->n) * es))
        fail(RS_EINVAL, "batched solves take device memory only (request " + std::to_string(i) +
                            " is a host pointer)");
    }
    solve_many(reqs, stream_of(opts));
    const auto done = record_completion(stream_of(opts));
    for (int i = 0; i < count; ++i) note_inflight(h[i], done);
    return RS_OK;
  });
}

rs_status rs_solve_ex(rs_handle h, void *B, int64_t ldb, int32_t nrhs,
                      const rs_options *opts) {
  return guarded([&]() -> rs_status {
    if (!h) fail(RS_EINVAL, "NULL handle");
    if (nrhs < 0) fail(RS_EINVAL, "nrhs must be >= 0");
    if (nrhs == 0) return RS_OK;
    if (!B) fail(RS_EINVAL, "NULL right-hand side");
    if (ldb < h->n) fail(RS_EINVAL, "ldb < n");
    const int mode = mode_of(opts);
    const hipStream_t st = stream_of(opts);
    const size_t es = h->cplx ? 16 : 8;
    const size_t span = ((size_t)(nrhs - 1) * (size_t)ldb + (size_t)h->n) * es;
    h->busy.fetch_add(1);
    struct Dec {
      rs_handle h;
      ~Dec() { h->busy.fetch_sub(1); }
    } dec{h};
    if (is_device_buffer(B, span)) {
      solve_one(h, B, ldb, nrhs, mode, st);
      note_inflight(h, st);
      return RS_OK;
    }
    // host right-hand sides: staged through device memory, synchronous
    const size_t col = (size_t)h->n * es;
    void *D = nullptr;
    RS_HIP_CHECK(hipMallocAsync(&D, col * (size_t)nrhs, st));
    struct Freer {
      void *p;
      hipStream_t st;
      ~Freer() {
        (void)hipFreeAsync(p, st);
        (void)hipStreamSynchronize(st);
      }
    } freer{D, st};
    RS_HIP_CHECK(hipMemcpy2DAsync(D, col, B, (size_t)ldb * es, col, (size_t)nrhs,
                                  hipMemcpyHostToDevice, st));
    solve_one(h, D, h->n, nrhs, mode, st);
    RS_HIP_CHECK(hipMemcpy2DAsync(B, (size_t)ldb * es, D, col, col, (size_t)nrhs,
                                  hipMemcpyDeviceToHost, st));
    RS_HIP_CHECK(hipStreamSynchronize(st));
    return RS_OK;
  });
}

rs_status rs_solve(rs_handle h, void *B, int64_t ldb, int32_t nrhs, void *stream) {
  rs_options o{RS_LAUNCH_LEVEL, stream};
  return rs_solve_ex(h, B, ldb, nrhs, &o);
}

rs_status rs_matvec(rs_handle h, const void *X, int64_t ldx, void *Y, int64_t ldy, int32_t nrhs,
                    void *stream) {
  return guarded([&]() -> rs_status {
    if (!h) fail(RS_EINVAL, "NULL handle");
    if (nrhs < 0) fail(RS_EINVAL, "nrhs must be >= 0");
    if (nrhs == 0) return RS_OK;
    if (!X || !Y) fail(RS_EINVAL, "NULL input or output");
    if (ldx < h->n || ldy < h->n) fail(RS_EINVAL, "ldx or ldy < n");
    const size_t es = h->cplx ? 16 : 8;
    const size_t sx = ((size_t)(nrhs - 1) * (size_t)ldx + (size_t)h->n) * es;
    const size_t sy = ((size_t)(nrhs - 1) * (size_t)ldy + (size_t)h->n) * es;
    if (!is_device_buffer(X, sx) || !is_device_buffer(Y, sy))
      fail(RS_EINVAL, "rs_matvec takes device memory only");
    const char *x0 = static_cast<const char *>(X), *y0 = static_cast<const char *>(Y);
    if (x0 < y0 + sy && y0 < x0 + sx) fail(RS_EINVAL, "X and Y overlap");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    h->busy.fetch_add(1);
    struct Dec {
      rs_handle h;
      ~Dec() { h->busy.fetch_sub(1); }
    } dec{h};
    matvec_one(h, X, ldx, Y, ldy, nrhs, st);
    note_inflight(h, st);
    return RS_OK;
  });
}

rs_status rs_solve_noalloc(rs_handle h, void *B, int64_t ldb, int32_t nrhs, void *stream) {
  return guarded([&]() -> rs_status {
    if (!h) fail(RS_EINVAL, "NULL handle");
    if (nrhs < 0) fail(RS_EINVAL, "nrhs must be >= 0");
    if (nrhs == 0) return RS_OK;
    if (!B) fail(RS_EINVAL, "NULL right-hand side");
    if (ldb < h->n) fail(RS_EINVAL, "ldb < n");
    const size_t es = h->cplx ? 2 : 1;
    if (!is_device_buffer(B, ((size_t)(nrhs - 1) * (size_t)ldb + (size_t)h->n) * es * 8))
      fail(RS_EINVAL, "rs_solve_noalloc takes device memory only");
    // workspace layout in the scratch array: W (n * nrhs scalars), then the wide-box
    // staging starting at the next 256-byte boundary
    const size_t cap = noalloc_scratch_bytes() / sizeof(double);
    const size_t w_doubles = (size_t)h->n * (size_t)nrhs * es;
    const size_t wide_off = (w_doubles + 31) & ~size_t(31);
    const int64_t wide_min = solve_wide_min_doubles(h, nrhs);
    const size_t need = wide_min > 0 ? wide_off + (size_t)wide_min : w_doubles;
    if (need > cap)
      fail(RS_EINVAL, "solve needs " + std::to_string(need * sizeof(double)) +
                          " bytes of scratch; rs_solve_noalloc is limited to " +
                          std::to_string(noalloc_scratch_bytes()) + " bytes per call");
    double *base = noalloc_scratch();
    const int64_t wide_sz =
        wide_min > 0 ? std::min<int64_t>(solve_wide_doubles(h, nrhs), (int64_t)(cap - wide_off)) : 0;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    h->busy.fetch_add(1);
    struct Dec {
      rs_handle h;
      ~Dec() { h->busy.fetch_sub(1); }
    } dec{h};
    {
      CaptureScope no_profiler_events;
      solve_one_into(h, B, ldb, nrhs, RS_LAUNCH_LEVEL, st, base, wide_sz > 0 ? base + wide_off : nullptr,
                     wide_sz);
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    RS_HIP_CHECK(hipStreamIsCapturing(st, &cs));
    if (cs == hipStreamCaptureStatusNone) note_inflight(h, st);
    return RS_OK;
  });
}

rs_status rs_plan_create(int32_t count, const rs_handle *h, void *const *B, const int64_t *ldb,
                         const int32_t *nrhs, rs_plan *out) {
  return guarded([&]() -> rs_status {
    if (!out) fail(RS_EINVAL, "NULL output");
    if (count < 1) fail(RS_EINVAL, "count must be >= 1");
    if (!h || !B || !ldb || !nrhs) fail(RS_EINVAL, "NULL argument");
    std::vector<SolveRequest> reqs(count);
    for (int i = 0; i < count; ++i) {
      if (!h[i]) fail(RS_EINVAL, "NULL handle");
      if (nrhs[i] < 1) fail(RS_EINVAL, "nrhs must be >= 1");
      if (!B[i]) fail(RS_EINVAL, "NULL right-hand side");
      if (ldb[i] < h[i]->n) fail(RS_EINVAL, "ldb < n");
      reqs[i] = SolveRequest{h[i], B[i], ldb[i], nrhs[i]};
    }
    require_device();
    *out = reinterpret_cast<rs_plan>(make_plan(reqs));
    return RS_OK;
  });
}

rs_status rs_plan_launch(rs_plan p, void *stream) {
  return guarded([&]() -> rs_status {
    if (!p) fail(RS_EINVAL, "NULL plan");
    launch_plan(reinterpret_cast<SolvePlan *>(p), static_cast<hipStream_t>(stream));
    return RS_OK;
  });
}

rs_status rs_plan_free(rs_plan p) {
  return guarded([&]() -> rs_status {
    if (!p) return RS_OK;
    RS_HIP_CHECK(hipDeviceSynchronize());
    delete reinterpret_cast<SolvePlan *>(p);
    return RS_OK;
  });
}

rs_status rs_autotune(rs_handle h, const int32_t *nrhs_list, int32_t count, int32_t reps,
                      void *stream) {
  return guarded([&]() -> rs_status {
    if (!h || !nrhs_list || count < 1) fail(RS_EINVAL, "NULL handle or empty nrhs list");
    if (reps < 1) fail(RS_EINVAL, "reps must be >= 1");
    std::vector<int> lst;
    for (int i = 0; i < count; ++i) {
      if (nrhs_list[i] < 1 || nrhs_list[i] > (1 << 16)) fail(RS_EINVAL, "nrhs out of range");
      lst.push_back(nrhs_list[i]);
    }
    h->busy.fetch_add(1);
    struct Dec {
      rs_handle h;
      ~Dec() { h->busy.fetch_sub(1); }
    } dec{h};
    autotune(h, lst, reps, static_cast<hipStream_t>(stream));
    return RS_OK;
  });
}

rs_status rs_tune_entries(uint32_t *keys, int32_t *widths, int32_t cap, int32_t *count) {
  return guarded([&]() -> rs_status {
    const auto e = tune_entries();
    if (count) *count = (int32_t)e.size();
    if ((keys || widths) && cap < (int32_t)e.size()) fail(RS_EINVAL, "buffer too small");
    for (size_t i = 0; i < e.size(); ++i) {
      if (keys) keys[i] = e[i].first;
      if (widths) widths[i] = e[i].second;
    }
    return RS_OK;
  });
}

rs_status rs_tune_clear(void) {
  return guarded([&]() -> rs_status {
    tune_clear();
    return RS_OK;
  });
}

rs_status rs_tune_save(const char *path) {
  return guarded([&]() -> rs_status {
    if (!path) fail(RS_EINVAL, "NULL path");
    tune_save(path);
    return RS_OK;
  });
}

rs_status rs_tune_load(const char *path) {
  return guarded([&]() -> rs_status {
    if (!path) fail(RS_EINVAL, "NULL path");
    tune_load(path);
    return RS_OK;
  });
}

rs_status rs_free(rs_handle h) {
  return guarded([&]() -> rs_status {
    if (!h) return RS_OK;
    if (h->busy.load() != 0) fail(RS_EBUSY, "handle is in use by a running call");
    if (has_inflight(h)) fail(RS_EBUSY, "solves on this handle are still queued or running");
    RS_HIP_CHECK(hipDeviceSynchronize());
    h->arena.release();                  // device memory back to the cache now
    Reaper::get().defer([h] { delete h; });   // host lists freed in the background
    return RS_OK;
  });
}

rs_status rs_query(rs_handle h, rs_stats *out) {
  return guarded([&]() -> rs_status {
    if (!h || !out) fail(RS_EINVAL, "NULL argument");
    *out = h->stats;
    return RS_OK;
  });
}

rs_status rs_factor_estimate(const rs_kernel *k, rs_tree t, double eps, size_t *resident,
                             size_t *transient) {
  return guarded([&]() -> rs_status {
    if (!k || !t || !resident || !transient) fail(RS_EINVAL, "NULL argument");
    if (!(eps >= 0.0)) fail(RS_EINVAL, "eps must be >= 0");
    const FootprintEstimate e = factor_footprint(*k, t->t, eps);
    *resident = e.resident;
    *transient = e.transient;
    return RS_OK;
  });
}

rs_status rs_query_levels(rs_handle h, rs_level_stats *out, int32_t cap, int32_t *count) {
  return guarded([&]() -> rs_status {
    if (!h || !count) fail(RS_EINVAL, "NULL argument");
    if (cap < 0 || (cap > 0 && !out)) fail(RS_EINVAL, "bad output buffer");
    *count = (int32_t)h->level_stats.size();
    for (int32_t i = 0; i < cap && i < *count; ++i) out[i] = h->level_stats[i];
    return RS_OK;
  });
}

rs_status rs_box_skeletons(rs_handle h, int32_t *k_out, int64_t *skel_out, int64_t cap,
                           int64_t *total) {
  return guarded([&]() -> rs_status {
    if (!h) fail(RS_EINVAL, "NULL handle");
    int64_t need = 0;
    for (int b = 0; b < h->nbox; ++b) need += (int64_t)h->box_skel[b].size();
    if (total) *total = need;
    if (skel_out && cap < need) fail(RS_EINVAL, "skeleton buffer too small");
    int64_t off = 0;
    for (int b = 0; b < h->nbox; ++b) {
      if (k_out) k_out[b] = h->box_k[b];
      if (skel_out)
        for (int32_t g : h->box_skel[b]) skel_out[off++] = g;
    }
    return RS_OK;
  });
}

rs_status rs_box_export(rs_handle h, int64_t b, int32_t *n_out, int32_t *k_out, int64_t *J_out,
                        double *T_out) {
  return guarded([&]() -> rs_status {
    if (!h) fail(RS_EINVAL, "NULL handle");
    if (b < 0 || b >= h->nbox) fail(RS_EINVAL, "box index out of range");
    const std::vector<int32_t> &J = h->box_J[b];
    const int n = (int)J.size();
    const int k = h->box_k[b] < 0 ? 0 : h->box_k[b];
    if (n_out) *n_out = n;
    if (k_out) *k_out = k;
    if (J_out)
      for (int i = 0; i < n; ++i) J_out[i] = J[i];
    if (T_out && k > 0 && n - k > 0)
      RS_HIP_CHECK(hipMemcpy(T_out, h->box_slot[b] + slot_T(k, n - k),
                             (size_t)k * (n - k) * sizeof(double) * (h->cplx ? 2 : 1),
                             hipMemcpyDeviceToHost));
    return RS_OK;
  });
}

rs_status rs_profile_enable(int32_t on) {
  return guarded([&]() -> rs_status {
    prof_enable(on != 0);
    return RS_OK;
  });
}

rs_status rs_profile_reset(void) {
  return guarded([&]() -> rs_status {
    prof_reset();
    return RS_OK;
  });
}

rs_status rs_profile_read(int32_t family, int64_t *launches, double *total_ms, double *flops,
                          double *bytes, double *entries) {
  return guarded([&]() -> rs_status {
    if (family < 0 || family >= RS_K_COUNT) fail(RS_EINVAL, "unknown kernel family");
    prof_read(family, launches, total_ms, flops, bytes, entries);
    return RS_OK;
  });
}

}  // extern "C"
