// Serving loop: factorizations stay resident in device memory; solve requests are
// batched continuously across handles and right-hand-side counts; factor requests are
// admitted against a device-memory budget and run concurrently with the solves.
//
// Threads
//   solve thread      drains the solve queue into batches (solve_many) and enqueues
//                     them alternately on two streams, so a new batch starts while the
//                     previous one is still on the device;
//   completion thread waits for each batch's event in order and stamps its requests'
//                     completion times (latency = completion - submission);
//   factor thread     admits queued factor requests in arrival order when their
//                     estimated footprint fits the free budget, and factors them on a
//                     third stream.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include "runtime.h"

namespace rs {

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Ticket {
  uint64_t id = 0;
  bool is_factor = false;
  bool done = false;
  rs_status status = RS_OK;
  std::string error;
  rs_handle handle = nullptr;     // factor result
  double t_submit = 0, t_start = 0, t_done = 0;
  int32_t nrhs = 0;
};

struct SolveItem {
  std::shared_ptr<Ticket> tk;
  SolveRequest req;
  hipEvent_t after = nullptr;     // recorded on the producer's stream at submission
};

struct FactorItem {
  std::shared_ptr<Ticket> tk;
  rs_kernel k;
  Tree tree;
  std::vector<double> points, weights, normals, curvature;
  double eps;
  size_t estimate;
  FootprintEstimate model;
  int corr_key = 0;
};

struct InFlight {
  hipEvent_t ev;
  std::vector<SolveItem> items;
};

}  // namespace

}  // namespace rs

struct rs_server_s {
  size_t budget = 0;
  int32_t max_batch_requests = 64;
  int32_t max_batch_rhs = 4096;
  std::mutex mu;
  std::condition_variable cv_solve, cv_factor, cv_done, cv_inflight;
  std::deque<rs::SolveItem> solve_q;
  std::deque<std::unique_ptr<rs::FactorItem>> factor_q;
  std::deque<rs::InFlight> inflight;
  std::unordered_map<uint64_t, std::shared_ptr<rs::Ticket>> tickets;
  std::unordered_map<rs_handle, size_t> resident;      // handles created by the server
  // footprint model corrections by (kernel, decades of eps): kept / predicted resident
  // bytes of the factorizations done so far (never below 1)
  std::map<int, double> footprint_corr;
  size_t resident_bytes = 0;
  size_t reserved_bytes = 0;
  uint64_t next_id = 1;
  bool stop = false;
  hipStream_t solve_stream[2] = {nullptr, nullptr};
  hipStream_t factor_stream = nullptr;
  int device = 0;
  std::thread solve_thr, done_thr, factor_thr;
  // statistics
  std::vector<double> solve_latency_ms;
  int64_t solves_done = 0, rhs_done = 0, factors_done = 0, rejected = 0, batches = 0;
  double first_submit = -1, last_done = 0;
  std::string fatal;
};

namespace rs {

namespace {

int footprint_key(const rs_kernel &k, double eps) {
  return k.kind * 100 + (int)std::lround(std::max(0.0, -std::log10(std::max(eps, 1e-16))));
}

// (caller holds s->mu)
size_t corrected_estimate(const rs_server_s *s, const FootprintEstimate &m, int key) {
  auto it = s->footprint_corr.find(key);
  const double c = it == s->footprint_corr.end() ? 1.0 : it->second;
  return (size_t)((double)m.resident * c) + m.transient;
}

size_t handle_bytes(rs_handle h) {
  size_t b = 0;
  for (const auto &c : h->arena.chunks) b += c->bytes;
  return b;
}

}  // namespace

// Rank model of a factorization's device footprint.  Prior ranks: a box at height
// h = maxdepth - depth keeps about c d^p g^h skeletons (d = decades of eps; 2D curves
// p = 1, g = 1.14; 3D surfaces p = 2, g = 2: a box's boundary grows like its side),
// never more than its active set; complex (oscillatory) kernels 1.5 times more.  The
// active set of a leaf is its points, of a parent its children's skeletons.  Resident:
// each box's slot (slot_bound(n) scalars) and the root's inverse (n^2); transient: the
// largest level's box workspaces (n^2 + 16 n scalars each) plus a fixed 64 MiB for the
// index pools, descriptors and allocation granularity.
FootprintEstimate factor_footprint(const rs_kernel &k, const Tree &t, double eps) {
  const bool cplx = k.kind == RS_HELM2D_CFIE || k.kind == RS_HELM3D_SL;
  const double es = cplx ? 2.0 : 1.0;
  const double dec = std::max(1.0, -std::log10(std::max(eps, 1e-16)));
  const bool d3 = t.dim == 3;
  const double base = 1.7 * (d3 ? dec * dec : dec) * (cplx ? 1.5 : 1.0);
  const double growth = d3 ? 2.0 : 1.14;
  const int nb = t.nbox();
  std::vector<double> kk(nb, 0.0);
  std::vector<double> lvl_work(t.maxdepth + 1, 0.0);
  double resident = 0.0;
  for (int d = t.maxdepth; d >= 0; --d) {
    for (int b : t.levels[d]) {
      double n = 0.0;
      if (t.is_leaf(b)) {
        n = (double)(t.end[b] - t.begin[b]);
      } else {
        for (int c = t.first_child[b]; c < t.first_child[b] + t.nchild[b]; ++c) n += kk[c];
      }
      lvl_work[d] += n * n + 16.0 * n;
      if (d == 0) {
        resident += n * n;
      } else {
        kk[b] = std::min(n, base * std::pow(growth, (double)(t.maxdepth - d)));
        resident += (double)slot_bound((int)std::ceil(n));
      }
    }
  }
  double transient = 0.0;
  for (double w : lvl_work) transient = std::max(transient, w);
  FootprintEstimate e;
  e.resident = (size_t)(resident * es * sizeof(double));
  e.transient = (size_t)(transient * es * sizeof(double)) + (size_t(64) << 20);
  return e;
}

namespace {

void fail_ticket(rs_server_s *s, const std::shared_ptr<Ticket> &tk, rs_status st,
                 const std::string &msg) {
  std::lock_guard<std::mutex> lock(s->mu);
  tk->status = st;
  tk->error = msg;
  tk->done = true;
  tk->t_done = now_ms();
  s->cv_done.notify_all();
}

void solve_loop(rs_server_s *s) {
  (void)hipSetDevice(s->device);
  int which = 0;
  for (;;) {
    std::vector<SolveItem> batch;
    {
      std::unique_lock<std::mutex> lock(s->mu);
      s->cv_solve.wait(lock, [&] { return s->stop || !s->solve_q.empty(); });
      if (s->stop && s->solve_q.empty()) return;
      // at most two batches on the device at once (one per stream)
      s->cv_inflight.wait(lock, [&] { return s->stop || s->inflight.size() < 2; });
      int64_t cols = 0;
      while (!s->solve_q.empty() && (int)batch.size() < s->max_batch_requests) {
        const SolveItem &it = s->solve_q.front();
        if (!batch.empty() && cols + it.req.nrhs > s->max_batch_rhs) break;
        cols += it.req.nrhs;
        batch.push_back(it);
        s->solve_q.pop_front();
      }
    }
    if (batch.empty()) continue;
    hipStream_t st = s->solve_stream[which];
    which ^= 1;
    std::vector<SolveRequest> reqs;
    const double t_start = now_ms();
    for (SolveItem &it : batch) {
      reqs.push_back(it.req);
      it.tk->t_start = t_start;
    }
    hipEvent_t ev = nullptr;
    rs_status fail_st = RS_OK;
    std::string fail_msg;
    try {
      // the batch starts after the work each producer had queued when it submitted
      for (SolveItem &it : batch)
        if (it.after) RS_HIP_CHECK(hipStreamWaitEvent(st, it.after, 0));
      solve_many(reqs, st);
      RS_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      RS_HIP_CHECK(hipEventRecord(ev, st));
    } catch (const DeviceError &e) {
      fail_st = RS_EDEVICE;
      fail_msg = e.what;
    } catch (const UserError &e) {
      fail_st = e.code;
      fail_msg = e.what;
    } catch (const std::bad_alloc &) {
      fail_st = RS_ENOMEM;
      fail_msg = "host allocation failed";
    } catch (const std::exception &e) {
      fail_st = RS_EDEVICE;
      fail_msg = e.what();
    } catch (...) {
      fail_st = RS_EDEVICE;
      fail_msg = "unknown error in the solve loop";
    }
    if (fail_st != RS_OK) {
      for (SolveItem &it : batch) {
        it.req.h->busy.fetch_sub(1);
        if (it.after) (void)hipEventDestroy(it.after);
        fail_ticket(s, it.tk, fail_st, fail_msg);
      }
      if (ev) (void)hipEventDestroy(ev);
      continue;
    }
    std::lock_guard<std::mutex> lock(s->mu);
    s->inflight.push_back(InFlight{ev, std::move(batch)});
    s->batches++;
    s->cv_done.notify_all();
  }
}

void done_loop(rs_server_s *s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    InFlight f;
    {
      std::unique_lock<std::mutex> lock(s->mu);
      s->cv_done.wait(lock, [&] { return s->stop || !s->inflight.empty(); });
      if (s->inflight.empty()) {
        if (s->stop) return;
        continue;
      }
      f.ev = s->inflight.front().ev;
    }
    const hipError_t e = hipEventSynchronize(f.ev);
    const double t = now_ms();
    std::lock_guard<std::mutex> lock(s->mu);
    InFlight done = std::move(s->inflight.front());
    s->inflight.pop_front();
    for (SolveItem &it : done.items) {
      it.req.h->busy.fetch_sub(1);
      if (it.after) (void)hipEventDestroy(it.after);
      it.tk->t_done = t;
      it.tk->done = true;
      if (e != hipSuccess) {
        it.tk->status = RS_EDEVICE;
        it.tk->error = hipGetErrorString(e);
      } else {
        s->solve_latency_ms.push_back(t - it.tk->t_submit);
        s->solves_done++;
        s->rhs_done += it.req.nrhs;
      }
    }
    s->last_done = t;
    (void)hipEventDestroy(done.ev);
    s->cv_done.notify_all();
    s->cv_inflight.notify_all();
  }
}

void factor_loop(rs_server_s *s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    std::unique_ptr<FactorItem> item;
    {
      std::unique_lock<std::mutex> lock(s->mu);
      s->cv_factor.wait(lock, [&] {
        if (s->stop) return true;
        if (s->factor_q.empty()) return false;
        const FactorItem &f = *s->factor_q.front();
        return s->resident_bytes + s->reserved_bytes + f.estimate <= s->budget;
      });
      if (s->stop) return;
      item = std::move(s->factor_q.front());
      s->factor_q.pop_front();
      s->reserved_bytes += item->estimate;
    }
    item->k.normals = item->normals.empty() ? nullptr : item->normals.data();
    item->k.curvature = item->curvature.empty() ? nullptr : item->curvature.data();
    item->tk->t_start = now_ms();
    rs_status st = RS_OK;
    std::string msg;
    std::vector<rs_factor_s *> out;
    try {
      std::vector<FactorRequest> reqs{
          {&item->k, &item->tree, item->points.data(), item->weights.data(), item->eps}};
      factor_many(reqs, RS_LAUNCH_LEVEL, s->factor_stream, out);
    } catch (const UserError &e) {
      st = e.code;
      msg = e.what;
    } catch (const DeviceError &e) {
      st = RS_EDEVICE;
      msg = e.what;
    } catch (const std::bad_alloc &) {
      st = RS_ENOMEM;
      msg = "host allocation failed";
    } catch (const std::exception &e) {
      st = RS_EDEVICE;
      msg = e.what();
    } catch (...) {
      st = RS_EDEVICE;
      msg = "unknown error in the factor loop";
    }
    std::lock_guard<std::mutex> lock(s->mu);
    s->reserved_bytes -= item->estimate;
    Ticket &tk = *item->tk;
    tk.status = st;
    tk.error = msg;
    tk.done = true;
    tk.t_done = now_ms();
    if (st == RS_OK) {
      tk.handle = out[0];
      const size_t b = handle_bytes(out[0]);
      s->resident[out[0]] = b;
      s->resident_bytes += b;
      s->factors_done++;
      // correct the model for later requests of the same kernel and eps decade
      const double ratio = (double)b / std::max<double>(1.0, (double)item->model.resident);
      auto it = s->footprint_corr.find(item->corr_key);
      const double prev = it == s->footprint_corr.end() ? ratio : it->second;
      s->footprint_corr[item->corr_key] = std::max(1.0, 0.5 * prev + 0.5 * ratio);
    }
    s->cv_done.notify_all();
    s->cv_factor.notify_all();
  }
}

}  // namespace

}  // namespace rs

using namespace rs;

extern "C" {

rs_status rs_server_create(const rs_server_opts *o, rs_server *out) {
  try {
    if (!o || !out) throw UserError{RS_EINVAL, "NULL argument"};
    if (o->hbm_budget == 0) throw UserError{RS_EINVAL, "hbm_budget must be positive"};
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
      throw UserError{RS_EDEVICE, "no HIP device available"};
    auto s = std::make_unique<rs_server_s>();
    s->budget = o->hbm_budget;
    if (o->max_batch_requests > 0) s->max_batch_requests = o->max_batch_requests;
    if (o->max_batch_rhs > 0) s->max_batch_rhs = o->max_batch_rhs;
    RS_HIP_CHECK(hipGetDevice(&s->device));
    for (auto &st : s->solve_stream) RS_HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    RS_HIP_CHECK(hipStreamCreateWithFlags(&s->factor_stream, hipStreamNonBlocking));
    rs_server_s *p = s.get();
    p->solve_thr = std::thread(solve_loop, p);
    p->done_thr = std::thread(done_loop, p);
    p->factor_thr = std::thread(factor_loop, p);
    *out = s.release();
    return RS_OK;
  } catch (const UserError &e) {
    set_error(e.what);
    return e.code;
  } catch (const DeviceError &e) {
    set_error(e.what);
    return RS_EDEVICE;
  } catch (const std::exception &e) {
    set_error(e.what());
    return RS_EDEVICE;
  }
}

rs_status rs_server_submit_factor(rs_server s, const rs_kernel *k, rs_tree t,
                                  const double *points, const double *weights, double eps,
                                  uint64_t *ticket) {
  if (!s || !k || !t || !points || !weights || !ticket) {
    set_error("NULL argument");
    return RS_EINVAL;
  }
  try {
    validate_kernel(k, t->t, points, weights, eps);
  } catch (const UserError &e) {
    set_error(e.what);
    return e.code;
  }
  auto item = std::make_unique<FactorItem>();
  item->k = *k;
  item->tree = t->t;
  const int64_t n = t->t.n;
  const int dim = t->t.dim;
  item->points.assign(points, points + n * dim);
  item->weights.assign(weights, weights + n);
  if (k->normals) item->normals.assign(k->normals, k->normals + n * dim);
  if (k->curvature) item->curvature.assign(k->curvature, k->curvature + n);
  item->eps = eps;
  item->model = factor_footprint(*k, t->t, eps);
  item->corr_key = footprint_key(*k, eps);
  {
    std::lock_guard<std::mutex> lock(s->mu);
    item->estimate = corrected_estimate(s, item->model, item->corr_key);
  }
  auto tk = std::make_shared<Ticket>();
  tk->is_factor = true;
  tk->t_submit = now_ms();
  item->tk = tk;
  std::lock_guard<std::mutex> lock(s->mu);
  tk->id = s->next_id++;
  s->tickets[tk->id] = tk;
  *ticket = tk->id;
  if (item->estimate > s->budget) {
    tk->status = RS_ENOMEM;
    tk->error = "factor footprint exceeds the server's memory budget";
    tk->done = true;
    tk->t_done = tk->t_submit;
    s->rejected++;
    return RS_OK;
  }
  s->factor_q.push_back(std::move(item));
  s->cv_factor.notify_all();
  return RS_OK;
}

rs_status rs_server_submit_solve(rs_server s, rs_handle h, void *B, int64_t ldb, int32_t nrhs,
                                 void *stream, uint64_t *ticket) {
  if (!s || !h || !ticket || nrhs < 1 || !B || ldb < h->n) {
    set_error("bad solve request (NULL argument, nrhs < 1 or ldb < n)");
    return RS_EINVAL;
  }
  hipEvent_t after = nullptr;
  try {
    RS_HIP_CHECK(hipSetDevice(s->device));
    const size_t es = h->cplx ? 16 : 8;
    if (!is_device_buffer(B, ((size_t)(nrhs - 1) * (size_t)ldb + (size_t)h->n) * es))
      throw UserError{RS_EINVAL, "the server solves device memory only (B is a host pointer)"};
    RS_HIP_CHECK(hipEventCreateWithFlags(&after, hipEventDisableTiming));
    RS_HIP_CHECK(hipEventRecord(after, static_cast<hipStream_t>(stream)));
  } catch (const UserError &e) {
    if (after) (void)hipEventDestroy(after);
    set_error(e.what);
    return e.code;
  } catch (const DeviceError &e) {
    if (after) (void)hipEventDestroy(after);
    set_error(e.what);
    return RS_EDEVICE;
  }
  auto tk = std::make_shared<Ticket>();
  tk->nrhs = nrhs;
  tk->t_submit = now_ms();
  h->busy.fetch_add(1);
  std::lock_guard<std::mutex> lock(s->mu);
  tk->id = s->next_id++;
  s->tickets[tk->id] = tk;
  *ticket = tk->id;
  if (s->first_submit < 0) s->first_submit = tk->t_submit;
  s->solve_q.push_back(SolveItem{tk, SolveRequest{h, B, ldb, nrhs}, after});
  s->cv_solve.notify_all();
  return RS_OK;
}

rs_status rs_server_poll(rs_server s, uint64_t ticket, int32_t timeout_ms, int32_t *done,
                         rs_status *status, rs_handle *factor_out) {
  if (!s || !done) {
    set_error("NULL argument");
    return RS_EINVAL;
  }
  std::unique_lock<std::mutex> lock(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) {
    set_error("unknown ticket");
    return RS_EINVAL;
  }
  std::shared_ptr<Ticket> tk = it->second;
  if (timeout_ms != 0 && !tk->done) {
    auto pred = [&] { return tk->done; };
    if (timeout_ms < 0) s->cv_done.wait(lock, pred);
    else s->cv_done.wait_for(lock, std::chrono::milliseconds(timeout_ms), pred);
  }
  *done = tk->done ? 1 : 0;
  if (tk->done) {
    if (status) *status = tk->status;
    if (factor_out) *factor_out = tk->handle;
    if (tk->status != RS_OK) set_error(tk->error);
    s->tickets.erase(ticket);
  }
  return RS_OK;
}

rs_status rs_server_release(rs_server s, rs_handle h) {
  if (!s || !h) {
    set_error("NULL argument");
    return RS_EINVAL;
  }
  {
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->resident.find(h);
    if (it == s->resident.end()) {
      set_error("handle was not created by this server");
      return RS_EINVAL;
    }
    if (h->busy.load() != 0) {
      set_error("handle has queued or running solves");
      return RS_EBUSY;
    }
    s->resident_bytes -= it->second;
    s->resident.erase(it);
  }
  rs_status st = rs_free(h);
  std::lock_guard<std::mutex> lock(s->mu);
  s->cv_factor.notify_all();
  return st;
}

rs_status rs_server_query(rs_server s, rs_server_stats *out) {
  if (!s || !out) {
    set_error("NULL argument");
    return RS_EINVAL;
  }
  std::lock_guard<std::mutex> lock(s->mu);
  rs_server_stats r{};
  r.solves_done = s->solves_done;
  r.rhs_done = s->rhs_done;
  r.factors_done = s->factors_done;
  r.rejected = s->rejected;
  r.batches = s->batches;
  r.resident_bytes = (int64_t)s->resident_bytes;
  r.queued_solves = (int64_t)s->solve_q.size();
  r.queued_factors = (int64_t)s->factor_q.size();
  std::vector<double> lat = s->solve_latency_ms;
  if (!lat.empty()) {
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double q) {
      const double pos = q * (lat.size() - 1);
      const size_t lo = (size_t)pos;
      const size_t hi = std::min(lo + 1, lat.size() - 1);
      return lat[lo] + (pos - lo) * (lat[hi] - lat[lo]);
    };
    r.p50_ms = pct(0.50);
    r.p99_ms = pct(0.99);
    r.mean_ms = 0;
    for (double v : lat) r.mean_ms += v;
    r.mean_ms /= lat.size();
  }
  if (s->first_submit >= 0 && s->last_done > s->first_submit)
    r.window_ms = s->last_done - s->first_submit;
  *out = r;
  return RS_OK;
}

rs_status rs_server_reset_stats(rs_server s) {
  if (!s) return RS_EINVAL;
  std::lock_guard<std::mutex> lock(s->mu);
  s->solve_latency_ms.clear();
  s->solves_done = s->rhs_done = s->factors_done = s->rejected = s->batches = 0;
  s->first_submit = -1;
  s->last_done = 0;
  return RS_OK;
}

void rs_server_destroy(rs_server s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lock(s->mu);
    // let queued solves finish; drop queued factor requests
    s->cv_done.wait(lock, [&] { return s->solve_q.empty() && s->inflight.empty(); });
    s->stop = true;
    s->cv_solve.notify_all();
    s->cv_factor.notify_all();
    s->cv_done.notify_all();
    s->cv_inflight.notify_all();
  }
  s->solve_thr.join();
  s->done_thr.join();
  s->factor_thr.join();
  for (auto &kv : s->resident) rs_free(kv.first);
  for (auto &st : s->solve_stream) (void)hipStreamDestroy(st);
  (void)hipStreamDestroy(s->factor_stream);
  delete s;
}

}  // extern "C"
