#include "profile.hpp"

namespace ptebd {

Profiler*& active_profiler() {
  thread_local Profiler* p = nullptr;
  return p;
}

hipEvent_t Profiler::get() {
  std::lock_guard<std::mutex> lk(mu);
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  PTEBD_HIP(hipEventCreate(&e));
  return e;
}

void Profiler::clear() {
  for (auto& r : recs) {
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
}

Profiler::~Profiler() {
  clear();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

ProfScope::ProfScope(int cls_, double flops_, hipStream_t s_) : p(active_profiler()), s(s_), cls(cls_), flops(flops_) {
  if (p) {
    a = p->get();
    PTEBD_HIP(hipEventRecord(a, s));
  }
}

ProfScope::~ProfScope() {
  if (p && a) {
    hipEvent_t b = p->get();
    if (hipEventRecord(b, s) == hipSuccess) {
      std::lock_guard<std::mutex> lk(p->mu);
      p->recs.push_back({cls, flops, a, b});
    }
  }
}

}  // namespace ptebd
