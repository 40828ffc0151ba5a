// Persistent host worker pool shared by the tree builder and the level planner.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace rs {

// Persistent pool of host worker threads for the level planner (created on first use,
// alive for the process).  parallel_for(n, f) runs f(i) for i in [0, n) in contiguous
// chunks on the calling thread plus the workers, and returns when all are done.
//
// Dispatch is one atomic word: (generation << 40) | (chunk count << 20) | next chunk.
// A job publishes a new generation; workers claim chunks with compare-and-swap on that
// word, so a worker still finishing one job can never take a chunk of the next.  Idle
// workers spin for kSpinUs before sleeping on a condition variable (a planner issues
// its parallel loops in bursts a few hundred microseconds apart; waking sleeping
// threads costs tens of microseconds per loop, while longer spins take the host's cores
// from the GPU runtime's own threads).
constexpr int kPlanThreads = 16;
constexpr int kSpinUs = 300;
class PlanPool {
 public:
  static PlanPool &get() {
    static PlanPool *p = new PlanPool();     // never destroyed: workers may outlive main
    return *p;
  }
  int workers() const { return (int)th_.size(); }
  // Wakes sleeping workers so that they spin again (for kSpinUs) without a job: a caller
  // about to issue parallel loops after a pause calls it before its serial preamble, so
  // the first loop does not wait for threads to be scheduled.
  void wake() {
    std::lock_guard<std::mutex> lk(mu_);
    if (sleepers_ > 0) {
      wakes_.fetch_add(1, std::memory_order_relaxed);
      cv_.notify_all();
    }
  }
  // Runs job(0..nchunks) on the caller plus the workers (nchunks < 2^20).  One job at a
  // time: a caller that finds the pool busy (another thread's job) runs all of its
  // chunks itself.
  void run(int nchunks, const std::function<void(int)> &job) {
    std::unique_lock<std::mutex> owner(run_mu_, std::try_to_lock);
    if (!owner.owns_lock() || nchunks >= (1 << 20)) {
      for (int c = 0; c < nchunks; ++c) job(c);
      return;
    }
    job_ = &job;
    pending_.store(nchunks, std::memory_order_relaxed);
    gen_ = (gen_ + 1) & 0xFFFFFF;
    slot_.store(pack(gen_, nchunks, 0), std::memory_order_release);
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (sleepers_ > 0) cv_.notify_all();
    }
    int c;
    while (claim(gen_, c)) {
      job(c);
      pending_.fetch_sub(1, std::memory_order_acq_rel);
    }
    while (pending_.load(std::memory_order_acquire) != 0) relax();
    job_ = nullptr;
  }

 private:
  static uint64_t pack(uint32_t g, int n, int next) {
    return ((uint64_t)g << 40) | ((uint64_t)n << 20) | (uint64_t)next;
  }
  static uint32_t gen_of(uint64_t v) { return (uint32_t)(v >> 40); }
  static void relax() { __builtin_ia32_pause(); }
  bool claim(uint32_t g, int &c) {
    uint64_t v = slot_.load(std::memory_order_acquire);
    while (true) {
      if (gen_of(v) != g) return false;
      const int n = (int)((v >> 20) & 0xFFFFF), next = (int)(v & 0xFFFFF);
      if (next >= n) return false;
      if (slot_.compare_exchange_weak(v, v + 1, std::memory_order_acq_rel)) {
        c = next;
        return true;
      }
    }
  }
  PlanPool() {
    const int n = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()),
                                          kPlanThreads) - 1;
    for (int i = 0; i < n; ++i) th_.emplace_back([this] { loop(); });
    for (auto &t : th_) t.detach();
  }
  void loop() {
    uint32_t seen = 0;
    while (true) {
      auto t0 = std::chrono::steady_clock::now();
      uint64_t v = slot_.load(std::memory_order_acquire);
      int spins = 0;
      while (gen_of(v) == seen) {
        if (++spins % 64 == 0 &&
            std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(kSpinUs)) {
          std::unique_lock<std::mutex> lk(mu_);
          ++sleepers_;
          const uint32_t w0 = wakes_.load(std::memory_order_relaxed);
          cv_.wait(lk, [&] {
            return gen_of(slot_.load(std::memory_order_acquire)) != seen ||
                   wakes_.load(std::memory_order_relaxed) != w0;
          });
          --sleepers_;
          t0 = std::chrono::steady_clock::now();     // spin again before the next sleep
        } else {
          relax();
        }
        v = slot_.load(std::memory_order_acquire);
      }
      seen = gen_of(v);
      int c;
      while (claim(seen, c)) {
        (*job_)(c);
        pending_.fetch_sub(1, std::memory_order_acq_rel);
      }
    }
  }
  std::vector<std::thread> th_;
  std::mutex run_mu_;      // held by the caller whose job the workers serve
  std::mutex mu_;          // sleeping workers
  std::condition_variable cv_;
  int sleepers_ = 0;
  uint32_t gen_ = 0;       // written by the run_mu_ holder only
  const std::function<void(int)> *job_ = nullptr;
  std::atomic<uint64_t> slot_{0};
  std::atomic<int> pending_{0};
  std::atomic<uint32_t> wakes_{0};
};

// Background release of large host structures made of many small allocations (the
// per-box lists of a factorization), off the caller's path.  One thread, created on
// first use, runs the deferred jobs in order; jobs still queued at process exit are
// dropped (their memory goes with the process).
class Reaper {
 public:
  static Reaper &get() {
    static Reaper *r = new Reaper();
    return *r;
  }
  void defer(std::function<void()> f) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      q_.push_back(std::move(f));
    }
    cv_.notify_one();
  }

 private:
  Reaper() { std::thread([this] { loop(); }).detach(); }
  void loop() {
    while (true) {
      std::function<void()> f;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return !q_.empty(); });
        f = std::move(q_.front());
        q_.pop_front();
      }
      f();
    }
  }
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::function<void()>> q_;
};

template <class F>
void parallel_for(int n, F &&f, int grain = 32) {
  PlanPool &pool = PlanPool::get();
  const int nt = std::max(1, std::min(pool.workers() + 1, n / grain));
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  const int nchunks = std::min(n, 4 * nt);
  const int chunk = (n + nchunks - 1) / nchunks;
  const std::function<void(int)> job = [&](int c) {
    for (int i = c * chunk; i < std::min(n, (c + 1) * chunk); ++i) f(i);
  };
  pool.run((n + chunk - 1) / chunk, job);
}

}  // namespace rs
