// Per-launch timing of the library's kernels with HIP events (opt-in).
#pragma once

#include <mutex>
#include <vector>

#include "common.hpp"

namespace ptebd {

enum KernelClass { K_GEMM_FP64 = 0, K_GEMM_FP32 = 1, K_HERM_EIG = 2, K_HERM_APPLY = 3, K_JAC_GRAM = 4,
                   K_JAC_ROTATE = 5, K_NCLASS = 6 };

struct Profiler {
  struct Rec {
    int cls;
    double flops;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  std::mutex mu;   // launchers of several worker threads report here
  hipEvent_t get();
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
  hipEvent_t a = nullptr;
  ProfScope(int cls_, double flops_, hipStream_t s_);
  ~ProfScope();
};

}  // namespace ptebd
