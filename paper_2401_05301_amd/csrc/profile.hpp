// Per-launch timing of the library's kernels with HIP events (opt-in).
#pragma once

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace ptebd {

enum KernelClass { K_GEMM_FP64 = 0, K_GEMM_FP32 = 1, K_HERM_EIG = 2, K_HERM_APPLY = 3, K_JAC_GRAM = 4,
                   K_JAC_ROTATE = 5, K_NCLASS = 6 };

// Launch records are folded into per-class totals as soon as their end
// event has completed, and the events go back to a pool, so a long profiled
// run holds a bounded number of events.
struct Profiler {
  struct Rec {
    int cls;
    double flops;
    hipEvent_t a, b;
    const char* tag;   // call site (string literal) or null
  };
  struct Tot {
    double ms = 0.0, flops = 0.0;
    int64_t launches = 0;
  };
  std::map<std::string, Tot> by_tag;   // totals per call site
  std::vector<Rec> recs;            // launches not folded yet
  std::vector<hipEvent_t> pool;     // idle events
  double ms[K_NCLASS] = {};
  double flops[K_NCLASS] = {};
  int64_t launches[K_NCLASS] = {};
  // Start and end of every folded launch (ms after origin, an event recorded
  // on the handle's stream when profiling was enabled, before any launch).
  hipEvent_t origin = nullptr;
  std::vector<std::pair<float, float>> spans[K_NCLASS];
  // Starts recording: clears the totals and records the origin on s.
  void start(hipStream_t s);
  // Milliseconds during which at least one launch of class cls ran (the
  // union of its folded spans).
  double busy_ms(int cls);
  std::mutex mu;   // launchers of several worker threads report here
  hipEvent_t get();
  void put(int cls, double flops, hipEvent_t a, hipEvent_t b, const char* tag);
  // Folds the finished records (every record when all_done: the caller has
  // synchronised every stream the records were made on).
  void fold(bool all_done);
  void clear();
  ~Profiler();
};

// The profiler the launchers of the calling thread report to (null: off).
Profiler*& active_profiler();

// Brackets one launch on stream s with a pair of events when profiling is on.
struct ProfScope {
  Profiler* p;
  hipStream_t s;
  int cls;
  double flops;
  const char* tag;
  hipEvent_t a = nullptr;
  ProfScope(int cls_, double flops_, hipStream_t s_, const char* tag_ = nullptr);
  ~ProfScope();
};

}  // namespace ptebd
