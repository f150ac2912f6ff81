#include "profile.hpp"

#include <algorithm>

namespace ptebd {

namespace {
// Pending records above which a new record triggers a fold of the finished ones.
constexpr size_t kFoldAt = 512;
}  // namespace

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

void Profiler::put(int cls, double fl, hipEvent_t a, hipEvent_t b, const char* tag) {
  bool full;
  {
    std::lock_guard<std::mutex> lk(mu);
    recs.push_back({cls, fl, a, b, tag});
    full = recs.size() >= kFoldAt;
  }
  if (full) fold(false);
}

void Profiler::fold(bool all_done) {
  std::lock_guard<std::mutex> lk(mu);
  size_t keep = 0;
  for (size_t i = 0; i < recs.size(); ++i) {
    Rec& r = recs[i];
    if (!all_done) {
      const hipError_t q = hipEventQuery(r.b);
      if (q == hipErrorNotReady) {
        // not an error: clear it from this thread's last-error slot, which
        // the launchers check after every launch
        (void)hipGetLastError();
        recs[keep++] = r;
        continue;
      }
      PTEBD_HIP(q);
    }
    float e = 0.f;
    PTEBD_HIP(hipEventElapsedTime(&e, r.a, r.b));
    if (origin) {
      float t0 = 0.f;
      PTEBD_HIP(hipEventElapsedTime(&t0, origin, r.a));
      spans[r.cls].push_back({t0, t0 + e});
    }
    ms[r.cls] += e;
    flops[r.cls] += r.flops;
    launches[r.cls] += 1;
    if (r.tag) {
      Tot& t = by_tag[r.tag];
      t.ms += e;
      t.flops += r.flops;
      t.launches += 1;
    }
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.resize(keep);
}

void Profiler::clear() {
  std::lock_guard<std::mutex> lk(mu);
  for (auto& r : recs) {
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
  for (int c = 0; c < K_NCLASS; ++c) {
    ms[c] = 0.0;
    flops[c] = 0.0;
    launches[c] = 0;
    spans[c].clear();
  }
  by_tag.clear();
  if (origin) pool.push_back(origin);
  origin = nullptr;
}

void Profiler::start(hipStream_t s) {
  clear();
  hipEvent_t o = get();
  PTEBD_HIP(hipEventRecord(o, s));
  std::lock_guard<std::mutex> lk(mu);
  origin = o;
}

double Profiler::busy_ms(int cls) {
  std::lock_guard<std::mutex> lk(mu);
  auto v = spans[cls];
  std::sort(v.begin(), v.end());
  double busy = 0.0, lo = 0.0, hi = -1.0;
  for (const auto& x : v) {
    if (x.first > hi) {
      if (hi > lo) busy += hi - lo;
      lo = x.first;
      hi = x.second;
    } else if (x.second > hi) {
      hi = x.second;
    }
  }
  if (hi > lo) busy += hi - lo;
  return busy;
}

Profiler::~Profiler() {
  clear();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

ProfScope::ProfScope(int cls_, double flops_, hipStream_t s_, const char* tag_)
    : p(active_profiler()), s(s_), cls(cls_), flops(flops_), tag(tag_) {
  if (p) {
    a = p->get();
    PTEBD_HIP(hipEventRecord(a, s));
  }
}

ProfScope::~ProfScope() {
  if (p && a) {
    hipEvent_t b = nullptr;
    try {
      b = p->get();
    } catch (...) {
      return;   // a destructor must not throw: the launch simply goes untimed
    }
    if (hipEventRecord(b, s) == hipSuccess) {
      try {
        p->put(cls, flops, a, b, tag);
      } catch (...) {
      }
    }
  }
}

}  // namespace ptebd
