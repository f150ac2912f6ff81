// Shared device/host helpers of the TEBD library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace ptebd {

// Error raised inside the library; converted to a tebd_status at the ABI.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define PTEBD_HIP(call)                                                               \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::ptebd::Error(-3, std::string(#call " failed: ") + hipGetErrorString(e_)); \
  } while (0)

#define PTEBD_LAUNCH_CHECK() PTEBD_HIP(hipGetLastError())

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Planar complex matrix view: element (i, j) at re[i*ld + j], im[i*ld + j].
struct ZMat {
  double* re;
  double* im;
  int64_t ld;
};

// Batched launches over independent matrices: the matrix that owns
// work-group bid, given first[i], the first work-group of matrix i
// (first[count] the total; every matrix has at least one work-group).
__device__ __forceinline__ int batch_owner(const int64_t* first, int count, int64_t bid) {
  int lo = 0, hi = count;   // first[lo] <= bid < first[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= bid)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Sets the thread-local message returned by tebd_last_error().
void set_last_error(const std::string& msg);

__host__ __device__ inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace ptebd
