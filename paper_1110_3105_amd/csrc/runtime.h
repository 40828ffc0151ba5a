// Host runtime: device arenas, factor handles, the level planner and the solve driver.
#pragma once

#include <atomic>
#include <functional>
#include <memory>
#include <mutex>
#include <vector>

#include "rs_internal.h"
#include "tree.h"

namespace rs {

// Owning device allocation.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // Grow-only; contents are not preserved when it grows.  Waits for the device first:
  // queued kernels may still read the old buffer.
  void ensure(size_t b) {
    if (b <= bytes) return;
    if (p) RS_HIP_CHECK(hipDeviceSynchronize());
    release();
    RS_HIP_CHECK(hipMalloc(&p, b < 256 ? 256 : b));
    bytes = b < 256 ? 256 : b;
  }
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// Bump allocator over device chunks; everything lives until the owner is freed.  Chunks
// come from (and return to) a process-wide cache of released chunks, so a factorization
// that follows a freed one reuses its device memory instead of hipFree + hipMalloc; the
// cache keeps at most kChunkCacheBytes.  Owners release an arena only once no queued
// work uses it (rs_free and the server's release wait for the device first).
constexpr size_t kChunkCacheBytes = size_t(2) << 30;
struct Arena {
  std::vector<std::unique_ptr<DevBuf>> chunks;
  size_t used = 0;
  size_t total = 0;
  void *alloc(size_t bytes);
  // Returns every chunk to the process-wide cache now (the owner must not use the
  // arena's memory afterwards).
  void release();
  template <class T> T *alloc_n(int64_t n) { return static_cast<T *>(alloc(sizeof(T) * (size_t)n)); }
  Arena() = default;
  Arena(const Arena &) = delete;
  Arena &operator=(const Arena &) = delete;
  ~Arena();
};

// One compressed level (or the root) of one factored problem.
struct LevelRec {
  int depth = 0;
  std::vector<int> boxes;
  std::vector<SweepBox> sweep;     // host copy (device pointers inside)
  SweepBox *d_sweep = nullptr;     // device copy
  int max_n = 0;
  int n_small = 0;                 // sweep[0, n_small): MFMA class (n <= kMfmaMaxN)
  int max_n_small = 0, max_n_large = 0;
  int max_k_large = 0, max_r_large = 0;   // over the wide class sweep[n_small, end)
  // Orders the boxes MFMA class (n <= mfma_limit) first and records the class boundary.
  void partition_classes(int mfma_limit);
};

// A completion event shared by the handles one call touched (destroyed with the last
// reference).
struct SharedEvent {
  hipEvent_t ev = nullptr;
  ~SharedEvent() {
    if (ev) (void)hipEventDestroy(ev);
  }
};

// Device descriptors of the compressed forward operator, built on a handle's first
// rs_matvec call (per compressed level, finest first, and the root).
struct MvLevel {
  MvBox *d = nullptr;
  int count = 0, max_k = 0, max_r = 0, max_n = 0;
};
struct MvPlan {
  std::vector<MvLevel> levels;
  MvLevel root;
  ProbDev *d_prob = nullptr;
  int64_t save_rows = 0;           // skeleton rows kept for the downward pass
};

}  // namespace rs

struct rs_factor_s {
  int dim = 0;
  int64_t n = 0;
  int kind = 0;
  bool cplx = false;                     // complex128 operator (Helmholtz)
  rs::Arena arena;                       // geometry, factors, index lists, descriptors
  int64_t *d_perm = nullptr;             // tree position -> caller index
  rs::ProbDev prob{};                    // device view of the geometry
  std::vector<rs::LevelRec> levels;      // compressed depths, finest first
  rs::LevelRec root;
  // host-side record for queries
  std::vector<int32_t> box_k;            // -1 for the root
  std::vector<std::vector<int32_t>> box_J, box_skel;
  std::vector<double *> box_slot;        // factor slot per box (scalars of the handle's type)
  int nbox = 0;
  rs_stats stats{};
  std::vector<rs_level_stats> level_stats;   // finest level first, the root last
  std::atomic<int> busy{0};
  std::mutex inflight_mu;
  std::vector<std::shared_ptr<rs::SharedEvent>> inflight;   // completions of enqueued solves
  // tree structure kept for the compressed forward operator (rs_matvec)
  std::vector<int32_t> tree_first_child, tree_nchild;
  std::vector<int64_t> tree_begin;
  std::mutex mv_mu;
  std::unique_ptr<rs::MvPlan> mv;
};

namespace rs {

struct FactorRequest {
  const rs_kernel *k;
  const Tree *tree;
  const double *points;
  const double *weights;
  double eps;
};

// Work queued on the factor's stream once a single problem's levels are factored and
// its roots launched (on another stream): it gets the handle, the stream and an event
// that completes with the roots, and must wait for that event before it reads them.
// The factorization then joins the roots and checks its errors.
using AfterRoots = std::function<void(rs_factor_s *, hipStream_t, hipEvent_t)>;

// Work a single-problem factorization interleaves with its own (each may be empty):
// begin -- on the side stream, once the geometry is on the device; level -- on the side
// stream, once a compressed level's factors are queued there and its solve descriptors
// uploaded; after_roots -- see AfterRoots.
struct FactorHooks {
  std::function<void(rs_factor_s *, hipStream_t)> begin;
  std::function<void(rs_factor_s *, const LevelRec &, hipStream_t)> level;
  AfterRoots after_roots;
};

// Factors every request; shared per-level launches across requests.  On success
// out[i] owns a new handle.  Throws on failure (all partial handles freed).
void factor_many(const std::vector<FactorRequest> &reqs, int launch_mode, hipStream_t st,
                 std::vector<rs_factor_s *> &out, const FactorHooks *hooks = nullptr);

// Factors one request and solves B (device, column-major, ldb >= n, nrhs columns) with
// it in the same call: the solve's permutation and upward sweeps run on the side stream
// as the levels complete, the rest after the roots.  The same bits as factor_many
// followed by solve_one.  Returns the new handle.
rs_factor_s *factor_and_solve(const FactorRequest &req, int launch_mode, hipStream_t st,
                              void *B, int64_t ldb, int nrhs);

// B: device, column-major, scalars of the handle's type (complex128 as re/im pairs).
void solve_one(rs_factor_s *h, void *B, int64_t ldb, int nrhs, int launch_mode,
               hipStream_t st, hipEvent_t roots_ready = nullptr);

// Y = A_eps X (the compressed forward operator of the handle's compression), X and Y
// device memory, column-major, caller order.  Enqueued on st.
void matvec_one(rs_factor_s *h, const void *X, int64_t ldx, void *Y, int64_t ldy, int nrhs,
                hipStream_t st);

// solve_one with caller-provided device workspace: W holds n * nrhs scalars of the
// handle's type; wide holds wide_sz doubles, at least solve_wide_min_doubles(h, nrhs)
// when that is positive (wide boxes are swept in chunks that fit).  Allocates nothing.
// roots_ready (optional): an event the stream waits for before the roots' step.
void solve_one_into(rs_factor_s *h, void *B, int64_t ldb, int nrhs, int launch_mode,
                    hipStream_t st, double *W, double *wide, int64_t wide_sz,
                    hipEvent_t roots_ready = nullptr);
// Smallest wide-class staging (doubles) a solve of nrhs columns can run with, and the
// size solve_one allocates (every wide box of a level at once, up to a cap).
int64_t solve_wide_min_doubles(const rs_factor_s *h, int nrhs);
int64_t solve_wide_doubles(const rs_factor_s *h, int nrhs);

// Device footprint of a factorization before it runs, from the tree, the kernel and eps
// (a rank model; the server corrects it by the bytes later factorizations kept).
struct FootprintEstimate {
  size_t resident = 0;     // bytes the handle keeps
  size_t transient = 0;    // bytes needed besides while it is factored
};
FootprintEstimate factor_footprint(const rs_kernel &k, const Tree &t, double eps);

// The allocation-free solve's device scratch (kernels.hip): a fixed array per device.
// noalloc_scratch() returns the current device's copy, looked up once per device.
size_t noalloc_scratch_bytes();
double *noalloc_scratch();

struct SolveRequest {
  rs_factor_s *h;
  void *B;
  int64_t ldb;
  int nrhs;
};
// Solves every request with shared per-level launches (levels aligned at the finest
// depth of each handle; all roots in one launch).  Enqueued on st; asynchronous.
void solve_many(const std::vector<SolveRequest> &reqs, hipStream_t st);

// A solve captured into a HIP graph: the launches of solve_many for fixed requests
// (handles, B buffers, nrhs), with a workspace and launch tables of its own.  Replaying
// it solves the current contents of the same B buffers; the handles stay busy until
// the plan is destroyed.
struct SolvePlan {
  std::vector<rs_factor_s *> handles;
  std::vector<void *> bufs;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~SolvePlan();
};
SolvePlan *make_plan(const std::vector<SolveRequest> &reqs);
void launch_plan(SolvePlan *p, hipStream_t st);

// Sweep tile-width autotuner (tune.cpp).
void autotune(rs_factor_s *h, const std::vector<int> &nrhs_list, int reps, hipStream_t st);
void tune_save(const char *path);
void tune_load(const char *path);

struct UserError {
  rs_status code;
  std::string what;
};

// True if p is device memory (or managed memory) of the current device; false for host
// memory (pageable, registered or pinned).  Throws UserError (RS_EINVAL) for device
// memory of another device, or when [p, p + bytes) runs past the end of p's device
// allocation (checked where the runtime reports the allocation's extent).
bool is_device_buffer(const void *p, size_t bytes);

// Solves issued on a handle: an event is recorded after each call on its stream, so
// that rs_free can tell whether any is still queued or running.  One event per call,
// shared by every handle the call touched.
std::shared_ptr<SharedEvent> record_completion(hipStream_t st);
void note_inflight(rs_factor_s *h, const std::shared_ptr<SharedEvent> &e);
void note_inflight(rs_factor_s *h, hipStream_t st);
// True if a recorded solve has not completed (completed events are released).
bool has_inflight(rs_factor_s *h);

// Argument checks shared by rs_factor and the server (throws UserError).
void validate_kernel(const rs_kernel *k, const Tree &t, const double *points,
                     const double *weights, double eps);

// ---- launch profiler (see rs_profile_enable)
struct Work {
  double flops = 0, bytes = 0, entries = 0;
  Work &operator+=(const Work &o) {
    flops += o.flops;
    bytes += o.bytes;
    entries += o.entries;
    return *this;
  }
};
bool prof_on();
// While alive on a thread, launches issued by that thread record no profiler events
// (stream capture: the graph holds kernel nodes only).
struct CaptureScope {
  CaptureScope();
  ~CaptureScope();
};
void prof_enable(bool on);
void prof_reset();
void prof_read(int family, int64_t *launches, double *ms, double *flops, double *bytes,
               double *entries);
void prof_add_work(int family, const Work &w);
// Brackets the launches issued during its lifetime with events on `st`.
class ProfScope {
 public:
  ProfScope(int family, hipStream_t st);
  ~ProfScope();
  ProfScope(const ProfScope &) = delete;
  ProfScope &operator=(const ProfScope &) = delete;

 private:
  int family_;
  hipStream_t st_;
  hipEvent_t start_ = nullptr, stop_ = nullptr;
  int device_ = 0;
  bool active_ = false;
};

// Algorithmic work of one box (counts documented with rs_profile_read).  For complex
// data a multiply-add counts 8 real flops and an entry 16 bytes.
Work work_assemble(int m, int n, bool cplx);
Work work_id(int m, int n, int k, bool cplx);
// Fused assembly + ID of a real box: the ID's flops, m n kernel entries, and the bytes of
// its outputs (R rows, T, skeleton order); the block itself never leaves the chip.
Work work_fused(int m, int n, int k);
Work work_factor(int n, int k, bool cplx);
Work work_sweep_up(int k, int r, int nrhs, bool cplx);
Work work_sweep_down(int k, int r, int nrhs, bool cplx);

}  // namespace rs
