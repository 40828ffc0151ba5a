// Launch profiler: HIP events on the launch stream around each kernel launch, plus
// the algorithmic work of the launch counted by the caller from the box sizes.
#include <algorithm>
#include <map>
#include <vector>

#include "runtime.h"

namespace rs {

namespace {

struct Pending {
  int family;
  int device;
  hipEvent_t start, stop;
};

struct Totals {
  int64_t launches = 0;
  double ms = 0, flops = 0, bytes = 0, entries = 0;
};

std::mutex g_prof_mutex;
std::atomic<bool> g_prof_on{false};
std::vector<Pending> g_pending;
Totals g_totals[RS_K_COUNT];
// events read by drain_locked, kept per device for later launches (creating an event
// allocates a signal: tens of microseconds per profiled launch otherwise)
std::map<int, std::vector<hipEvent_t>> g_free_events;

hipEvent_t take_event(int device) {
  {
    std::lock_guard<std::mutex> lock(g_prof_mutex);
    std::vector<hipEvent_t> &f = g_free_events[device];
    if (!f.empty()) {
      hipEvent_t e = f.back();
      f.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  RS_HIP_CHECK(hipEventCreate(&e));
  return e;
}

void drain_locked() {
  for (Pending &p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.stop) == hipSuccess &&
        hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      Totals &t = g_totals[p.family];
      t.launches += 1;
      t.ms += ms;
    }
    std::vector<hipEvent_t> &f = g_free_events[p.device];
    f.push_back(p.start);
    f.push_back(p.stop);
  }
  g_pending.clear();
}

}  // namespace

bool prof_on() { return g_prof_on.load(std::memory_order_relaxed); }

namespace {
thread_local int t_capture_depth = 0;
}
CaptureScope::CaptureScope() { ++t_capture_depth; }
CaptureScope::~CaptureScope() { --t_capture_depth; }

ProfScope::ProfScope(int family, hipStream_t st) : family_(family), st_(st) {
  if (!prof_on() || t_capture_depth > 0) return;
  RS_HIP_CHECK(hipGetDevice(&device_));
  start_ = take_event(device_);
  stop_ = take_event(device_);
  RS_HIP_CHECK(hipEventRecord(start_, st_));
  active_ = true;
}

ProfScope::~ProfScope() {
  if (!active_) return;
  (void)hipEventRecord(stop_, st_);
  std::lock_guard<std::mutex> lock(g_prof_mutex);
  g_pending.push_back({family_, device_, start_, stop_});
}

void prof_add_work(int family, const Work &w) {
  if (!prof_on()) return;
  std::lock_guard<std::mutex> lock(g_prof_mutex);
  Totals &t = g_totals[family];
  t.flops += w.flops;
  t.bytes += w.bytes;
  t.entries += w.entries;
}

// Complex data: a multiply-add is 8 real flops (4 for real data counted as 2 below, so
// the factor is 4) and an entry occupies 16 bytes.
static double flop_scale(bool cplx) { return cplx ? 4.0 : 1.0; }
static double byte_size(bool cplx) { return cplx ? 16.0 : 8.0; }

Work work_assemble(int m, int n, bool cplx) {
  Work w;
  w.entries = (double)m * n;
  w.bytes = byte_size(cplx) * m * n;
  return w;
}

// Algorithmic count of the ID by column-pivoted Householder QR stopped after k steps:
// sum over steps j < k of 4 (m - j)(n - j) flops (reflector applied to the remaining
// columns), i.e. 4mnk - 2k^2(m + n) + 4k^3/3, plus k^2 r for T = R11^{-1} R12
// (r = n - k).  The column norms the kernels recompute after every reflection (about
// 2 (m - j)(n - j) more per step) are implementation overhead and are not counted.
Work work_id(int m, int n, int k, bool cplx) {
  Work w;
  const double mm = m, nn = n, kk = k, r = n - k;
  const double f = 4.0 * mm * nn * kk - 2.0 * kk * kk * (mm + nn) + 4.0 * kk * kk * kk / 3.0 +
                   kk * kk * r;
  w.flops = std::max(f, 0.0) * flop_scale(cplx);
  w.bytes = byte_size(cplx) * (mm * nn + kk * r) + 4.0 * nn;
  return w;
}

Work work_fused(int m, int n, int k) {
  Work w = work_id(m, n, k, false);
  w.entries = (double)m * n;
  w.bytes = 8.0 * ((double)k * n + (double)k * (n - k)) + 4.0 * n;
  return w;
}

Work work_factor(int n, int k, bool cplx) {
  const double r = n - k, kk = k, nn = n;
  Work w;
  w.flops = (4.0 * nn * r * kk + 2.0 * r * r * r + 4.0 * r * r * kk + 2.0 * kk * kk * r) *
            flop_scale(cplx);
  w.entries = nn * nn;
  w.bytes = byte_size(cplx) * (3.0 * kk * r + r * r + kk * kk + kk * r);
  return w;
}

Work work_sweep_up(int k, int r, int nrhs, bool cplx) {
  Work w;
  const double ops = (double)r * r + 2.0 * k * r;
  w.flops = 2.0 * nrhs * ops * flop_scale(cplx);
  w.bytes = byte_size(cplx) * (ops + 2.0 * (k + r) * (double)nrhs);
  return w;
}

Work work_sweep_down(int k, int r, int nrhs, bool cplx) {
  Work w;
  const double ops = 2.0 * k * r;
  w.flops = 2.0 * nrhs * ops * flop_scale(cplx);
  w.bytes = byte_size(cplx) * (ops + 2.0 * (k + r) * (double)nrhs);
  return w;
}

void prof_enable(bool on) { g_prof_on.store(on); }

void prof_reset() {
  std::lock_guard<std::mutex> lock(g_prof_mutex);
  drain_locked();
  for (Totals &t : g_totals) t = Totals();
}

void prof_read(int family, int64_t *launches, double *ms, double *flops, double *bytes,
               double *entries) {
  std::lock_guard<std::mutex> lock(g_prof_mutex);
  drain_locked();
  const Totals &t = g_totals[family];
  if (launches) *launches = t.launches;
  if (ms) *ms = t.ms;
  if (flops) *flops = t.flops;
  if (bytes) *bytes = t.bytes;
  if (entries) *entries = t.entries;
}

}  // namespace rs
