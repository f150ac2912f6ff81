// tebd_diag_svd_noalloc: the truncated SVD of tebd_diag_svd with every
// device buffer carved from one file-scope array instead of hipMalloc.
//
// Each GPU the library runs on holds its own copy of `scratch` until the
// process ends.  Host code never names the array directly (its host-side
// symbol is not a device address): the device address is looked up once
// per device with hipGetSymbolAddress and kept in g_scratch.  Calls on one
// GPU share the array, so overlapping calls on the same GPU race; every
// value a call reads is written by that call first (the ledger and the
// counters are cleared with fill kernels).
#include <cstring>
#include <mutex>

#include "../../include/ptebd_diag.h"
#include "engine.hpp"

namespace {

constexpr int kMaxSide = 512;                 // m, n <= 512
constexpr int64_t kMaxElems = 65536;          // m * n <= 2^16 complex entries
constexpr int64_t kScratchDoubles = 1 << 20;  // 8 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use,
// with the device current).
double* scratch_ptr() {
  int dev = 0;
  PTEBD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw ptebd::Error(TEBD_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    PTEBD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw ptebd::Error(TEBD_EDEVICE, "scratch array has no device address");
    g_scratch[dev] = static_cast<double*>(p);
  }
  return g_scratch[dev];
}

// Bump allocator over the scratch array, 256-byte aligned pieces.
struct Carve {
  double* base;
  int64_t used = 0;
  double* take(int64_t n) {
    n = (std::max<int64_t>(n, 1) + 31) / 32 * 32;
    if (used + n > kScratchDoubles) throw ptebd::Error(TEBD_EINVAL, "noalloc SVD: scratch array too small");
    double* p = base + used;
    used += n;
    return p;
  }
  tebd_mps::Z z(int64_t n) {
    tebd_mps::Z q;
    q.re = take(n);
    q.im = take(n);
    return q;
  }
};

}  // namespace

extern "C" tebd_status tebd_diag_svd_noalloc(int32_t variant, int32_t m, int32_t n, const double* A, int32_t chi_max,
                                             double w_max, double eps, int32_t* k, double* s, double* vh, double* nrm,
                                             double* w, int32_t* sweeps) {
  if (m < 1 || n < 1 || !A || !k || !s || !vh || !nrm || !w || !sweeps || chi_max < 1) return TEBD_EINVAL;
  if (variant < TEBD_SVD_JACOBI || variant > TEBD_SVD_RANDOMIZED) return TEBD_EINVAL;
  if (m > kMaxSide || n > kMaxSide || (int64_t)m * n > kMaxElems) {
    ptebd::set_last_error("tebd_diag_svd_noalloc: m and n must be <= 512 and m * n <= 65536 (the scratch array "
                          "holds 8 MiB per device)");
    return TEBD_EINVAL;
  }
  if (!(eps >= 0.0) || !(w_max >= 0.0)) return TEBD_EINVAL;
  if (variant != TEBD_SVD_JACOBI && !(eps >= TEBD_GRAM_EPS_MIN)) {
    ptebd::set_last_error("the Gram route needs eps >= TEBD_GRAM_EPS_MIN (1e-6)");
    return TEBD_EINVAL;
  }
  try {
    Carve c{scratch_ptr()};
    tebd_mps M;   // settings and buffer pointers only: nothing here allocates
    M.stream = nullptr;
    M.opts.svd = variant;
    M.opts.trunc_weight = w_max;
    M.opts.trunc_rel = eps;
    M.opts.max_sweeps = 60;
    M.chi_max = chi_max;
    const int64_t r = std::min(m, n), mx = std::max(m, n);
    tebd_mps::Z a = c.z((int64_t)m * n), x = c.z((int64_t)m * n), vho = c.z(r * n);
    M.G = c.z(r * r);
    M.W = c.z(r * r);
    M.g_cap = r * r;
    M.norms = c.take(mx);
    M.inv_sig = c.take(mx);
    M.sq = c.take(mx);
    M.perm = reinterpret_cast<int*>(c.take(mx / 2 + 1));
    M.flags = reinterpret_cast<int*>(c.take(mx / 2 + 1));
    M.flags_cap = mx;
    const int64_t nbk = (r + 15) / 16 + 2;
    M.part_cap = (nbk / 2 + 1) * 16 * 1536;
    M.part = c.take(M.part_cap);
    M.info_i = reinterpret_cast<int*>(c.take(4));
    M.info_d = c.take(16);
    M.counter = reinterpret_cast<unsigned int*>(c.take(2));
    M.ledger = c.take(1);
    double* lam_out = c.take(r);
    // host mirrors of the read-backs: plain host memory of this call
    unsigned int h_counter[16] = {};
    int h_info[16] = {};
    double h_part[256] = {};
    M.h_counter = h_counter;
    M.h_info = h_info;
    M.h_part = h_part;
    PTEBD_HIP(hipMemcpy(a.re, A, sizeof(double) * m * n, hipMemcpyHostToDevice));
    PTEBD_HIP(hipMemcpy(a.im, A + (int64_t)m * n, sizeof(double) * m * n, hipMemcpyHostToDevice));
    // the array keeps the previous call's contents: the ledger starts at zero
    ptebd::fill_zero(M.ledger, 1, M.stream);
    ptebd::SvdIn in{a.re, a.im, n, m, n, nullptr, 1};
    const int kk = ptebd::svd_trunc(&M, in, lam_out, vho.re, vho.im, 0, x);
    PTEBD_HIP(hipStreamSynchronize(M.stream));
    double info[2];
    PTEBD_HIP(hipMemcpy(info, M.info_d, sizeof(double) * 2, hipMemcpyDeviceToHost));
    PTEBD_HIP(hipMemcpy(s, lam_out, sizeof(double) * kk, hipMemcpyDeviceToHost));
    PTEBD_HIP(hipMemcpy(vh, vho.re, sizeof(double) * kk * n, hipMemcpyDeviceToHost));
    PTEBD_HIP(hipMemcpy(vh + (int64_t)kk * n, vho.im, sizeof(double) * kk * n, hipMemcpyDeviceToHost));
    *k = kk;
    *nrm = info[0];
    *w = info[1];
    *sweeps = (int32_t)M.last_sweeps;
    // the struct must not release what it does not own
    M.h_counter = nullptr;
    M.h_info = nullptr;
    M.h_part = nullptr;
    return TEBD_OK;
  } catch (const ptebd::Error& e) {
    ptebd::set_last_error(e.what());
    return (tebd_status)e.code;
  }
}
