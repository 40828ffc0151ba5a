// Autotuner of the solve sweeps' tile widths.
//
// For each requested nrhs, the MFMA-class boxes of every level of a handle (and of its
// root) are swept with each valid tile width (16, 32, 64 columns per workgroup), timed
// with HIP events on the caller's stream; the times are summed per bucket of the tuning
// table (scalar type, ceil(log2 nrhs), largest box in steps of 32) and the fastest width
// of each bucket is recorded.  Widths change only the work distribution, never a result.
// Wide-class boxes have no width to choose (one 16 x 16 tile per wave).
#include <cstdio>
#include <map>

#include "runtime.h"

namespace rs {

void autotune(rs_factor_s *h, const std::vector<int> &nrhs_list, int reps, hipStream_t st) {
  const bool cplx = h->cplx;
  const int es = cplx ? 2 : 1;
  std::map<uint32_t, std::map<int, double>> acc;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  RS_HIP_CHECK(hipEventCreate(&ev0));
  RS_HIP_CHECK(hipEventCreate(&ev1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{ev0, ev1};
  CaptureScope quiet;     // no profiler events for the trial launches
  for (int nrhs : nrhs_list) {
    DevBuf W;
    W.ensure((size_t)h->n * nrhs * sizeof(double) * es);
    RS_HIP_CHECK(hipMemsetAsync(W.p, 0, W.bytes, st));
    double *w = W.as<double>();
    auto time_level = [&](const LevelRec &lv) {
      {
        const int cnt = lv.n_small, mx = lv.max_n_small;
        if (cnt <= 0) return;
        const uint32_t key = tune_key(true, es, nrhs, mx);
        static const int cands[] = {16, 32, 64};
        for (int nt : cands) {
          if (!sweep_nt_valid(true, nt, mx, es)) continue;
          auto run = [&](bool up) {
            launch_sweep_mfma(cplx, up, lv.d_sweep, 0, cnt, w, nrhs, mx, st, nt);
          };
          run(true);                                   // warm-up
          RS_HIP_CHECK(hipEventRecord(ev0, st));
          for (int r = 0; r < reps; ++r) {
            run(true);
            run(false);
          }
          RS_HIP_CHECK(hipEventRecord(ev1, st));
          RS_HIP_CHECK(hipEventSynchronize(ev1));
          float ms = 0.0f;
          RS_HIP_CHECK(hipEventElapsedTime(&ms, ev0, ev1));
          acc[key][nt] += ms;
        }
      }
    };
    for (const LevelRec &lv : h->levels) time_level(lv);
    time_level(h->root);
    RS_HIP_CHECK(hipStreamSynchronize(st));
  }
  for (const auto &kv : acc) {
    int best = 0;
    double bt = 0.0;
    for (const auto &c : kv.second)
      if (best == 0 || c.second < bt) {
        best = c.first;
        bt = c.second;
      }
    if (best) tune_set(kv.first, best);
  }
}

void tune_save(const char *path) {
  FILE *f = std::fopen(path, "w");
  if (!f) throw UserError{RS_EINVAL, std::string("cannot write ") + path};
  std::fprintf(f, "# rs sweep tile widths: bucket-key width\n");
  for (const auto &e : tune_entries()) std::fprintf(f, "%u %d\n", e.first, e.second);
  std::fclose(f);
}

void tune_load(const char *path) {
  FILE *f = std::fopen(path, "r");
  if (!f) throw UserError{RS_EINVAL, std::string("cannot read ") + path};
  char line[256];
  std::vector<std::pair<uint32_t, int>> got;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    unsigned key = 0;
    int nt = 0;
    if (std::sscanf(line, "%u %d", &key, &nt) != 2) {
      std::fclose(f);
      throw UserError{RS_EINVAL, "malformed tuning file"};
    }
    const bool ok = (key & 1u) && (nt == 16 || nt == 32 || nt == 64);
    if (!ok) {
      std::fclose(f);
      throw UserError{RS_EINVAL, "tuning file names an invalid tile width"};
    }
    got.emplace_back(key, nt);
  }
  std::fclose(f);
  for (const auto &e : got) tune_set(e.first, e.second);
}

}  // namespace rs
