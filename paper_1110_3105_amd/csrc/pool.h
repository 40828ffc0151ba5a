// Persistent host worker pool shared by the tree builder and the level planner.
#pragma once

#include <algorithm>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace rs {

// Persistent pool of host worker threads for the level planner (created on first use,
// alive for the process).  parallel_for(n, f) runs f(i) for i in [0, n) in contiguous
// chunks on the calling thread plus the workers, and returns when all are done.
constexpr int kPlanThreads = 16;
class PlanPool {
 public:
  static PlanPool &get() {
    static PlanPool *p = new PlanPool();     // never destroyed: workers may outlive main
    return *p;
  }
  int workers() const { return (int)th_.size(); }
  // Runs job(0..nchunks) on the caller plus the workers.  One job at a time: a caller
  // that finds the pool busy (another thread's job) runs all of its chunks itself.
  void run(int nchunks, const std::function<void(int)> &job) {
    std::unique_lock<std::mutex> owner(run_mu_, std::try_to_lock);
    if (!owner.owns_lock()) {
      for (int c = 0; c < nchunks; ++c) job(c);
      return;
    }
    std::unique_lock<std::mutex> lk(mu_);
    job_ = &job;
    nchunks_ = nchunks;
    next_ = 1;                 // chunk 0 runs on the caller
    pending_ = nchunks - 1;
    ++gen_;
    cv_.notify_all();
    lk.unlock();
    job(0);
    lk.lock();
    while (true) {             // the caller helps with the remaining chunks
      if (next_ < nchunks_) {
        const int c = next_++;
        lk.unlock();
        job(c);
        lk.lock();
        --pending_;
        continue;
      }
      break;
    }
    done_cv_.wait(lk, [&] { return pending_ == 0; });
    job_ = nullptr;
  }

 private:
  PlanPool() {
    const int n = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()),
                                          kPlanThreads) - 1;
    for (int i = 0; i < n; ++i) th_.emplace_back([this] { loop(); });
    for (auto &t : th_) t.detach();
  }
  void loop() {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      cv_.wait(lk, [&] { return gen_ != seen; });
      seen = gen_;
      while (job_ && next_ < nchunks_) {
        const int c = next_++;
        const std::function<void(int)> *job = job_;
        lk.unlock();
        (*job)(c);
        lk.lock();
        if (--pending_ == 0) done_cv_.notify_all();
      }
    }
  }
  std::vector<std::thread> th_;
  std::mutex run_mu_;      // held by the caller whose job the workers serve
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)> *job_ = nullptr;
  int nchunks_ = 0, next_ = 0, pending_ = 0;
  uint64_t gen_ = 0;
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
