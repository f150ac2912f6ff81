// Diagnostic entry points (include/ptebd_diag.h): one kernel family at a time.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ptebd_diag.h"
#include "engine.hpp"

namespace {


struct Scratch {
  std::vector<void*> ptrs;
  double* alloc(int64_t n) {
    void* p = nullptr;
    PTEBD_HIP(hipMalloc(&p, sizeof(double) * std::max<int64_t>(n, 1)));
    ptrs.push_back(p);
    return static_cast<double*>(p);
  }
  double* upload(const double* h, int64_t n) {
    double* d = alloc(n);
    PTEBD_HIP(hipMemcpy(d, h, sizeof(double) * n, hipMemcpyHostToDevice));
    return d;
  }
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

}  // namespace

extern "C" tebd_status tebd_diag_zgemm(int32_t prec, int32_t m, int32_t n, int32_t k, int32_t transA, int32_t transB,
                                       const double* A, const double* B, const double* k_scale,
                                       const double* row_scale, const double* col_scale, int32_t herm,
                                       double* C) {
  if (m < 1 || n < 1 || k < 1 || !A || !B || !C || prec < 0 || prec > 2) return TEBD_EINVAL;
  try {
    Scratch sc;
    const int64_t na = (int64_t)m * k, nb = (int64_t)k * n, nc = (int64_t)m * n;
    double* a = sc.upload(A, 2 * na);
    double* b = sc.upload(B, 2 * nb);
    double* c = sc.alloc(2 * nc);
    ptebd::ZGemmArgs g;
    g.m = m; g.n = n; g.k = k;
    g.ar = a; g.ai = a + na; g.lda = transA ? m : k; g.transA = transA;
    g.br = b; g.bi = b + nb; g.ldb = transB ? k : n; g.transB = transB;
    g.cr = c; g.ci = c + nc; g.ldc = n;
    if (k_scale) g.k_scale = sc.upload(k_scale, k);
    if (row_scale) g.row_scale = sc.upload(row_scale, m);
    if (col_scale) g.col_scale = (herm && row_scale) ? g.row_scale : sc.upload(col_scale, n);
    g.herm_out = herm ? 1 : 0;
    ptebd::zgemm(g, prec, nullptr);
    PTEBD_HIP(hipDeviceSynchronize());
    PTEBD_HIP(hipMemcpy(C, c, sizeof(double) * 2 * nc, hipMemcpyDeviceToHost));
    return TEBD_OK;
  } catch (const ptebd::Error& e) {
    ptebd::set_last_error(e.what());
    return (tebd_status)e.code;
  }
}

extern "C" tebd_status tebd_diag_svd(int32_t variant, int32_t m, int32_t n, const double* A, int32_t chi_max,
                                     double w_max, double eps, int32_t* k, double* s, double* vh, double* nrm,
                                     double* w, int32_t* sweeps) {
  if (m < 1 || n < 1 || !A || !k || !s || !vh || !nrm || !w || !sweeps || chi_max < 1) return TEBD_EINVAL;
  if (variant < TEBD_SVD_JACOBI || variant > TEBD_SVD_RANDOMIZED) return TEBD_EINVAL;
  if (std::min(m, n) > 8192) return TEBD_EINVAL;
  if (!(eps >= 0.0) || !(w_max >= 0.0)) return TEBD_EINVAL;
  if (variant != TEBD_SVD_JACOBI && !(eps >= TEBD_GRAM_EPS_MIN)) {
    ptebd::set_last_error("the Gram route needs eps >= TEBD_GRAM_EPS_MIN (1e-6)");
    return TEBD_EINVAL;
  }
  tebd_mps M;
  try {
    PTEBD_HIP(hipStreamCreateWithFlags(&M.stream, hipStreamNonBlocking));
    M.own_stream = true;
    M.opts.svd = variant;
    M.opts.trunc_weight = w_max;
    M.opts.trunc_rel = eps;
    M.opts.max_sweeps = 60;
    M.chi_max = chi_max;
    const int64_t r = std::min(m, n), mx = std::max(m, n);
    auto z = [&](int64_t cnt) {
      tebd_mps::Z q;
      q.re = static_cast<double*>(ptebd::dev_alloc(&M, sizeof(double) * cnt));
      q.im = static_cast<double*>(ptebd::dev_alloc(&M, sizeof(double) * cnt));
      return q;
    };
    tebd_mps::Z a = z((int64_t)m * n), x = z((int64_t)m * n), vho = z(r * n);
    M.G = z(r * r);
    M.W = z(r * r);
    M.g_cap = r * r;
    M.norms = static_cast<double*>(ptebd::dev_alloc(&M, sizeof(double) * mx));
    M.inv_sig = static_cast<double*>(ptebd::dev_alloc(&M, sizeof(double) * mx));
    M.sq = static_cast<double*>(ptebd::dev_alloc(&M, sizeof(double) * mx));
    M.perm = static_cast<int*>(ptebd::dev_alloc(&M, sizeof(int) * mx));
    M.flags = static_cast<int*>(ptebd::dev_alloc(&M, sizeof(int) * mx));
    const int sp = ptebd::subspace_width((int)r, chi_max);
    if (variant != TEBD_SVD_JACOBI && sp > 0) {
      M.sub_p = sp;
      M.sub_r = (int)r;
      M.sZ = z((int64_t)sp * r);
      M.sY = z((int64_t)sp * r);
      M.sZ2 = z((int64_t)sp * r);
      M.sY2 = z((int64_t)sp * r);
      M.sH = z((int64_t)sp * sp);
      M.sW = z((int64_t)sp * sp);
      M.nY = z((int64_t)sp * sp);
      M.nZ = z((int64_t)sp * sp);
      M.nY2 = z((int64_t)sp * sp);
      M.nZ2 = z((int64_t)sp * sp);
      M.ns_part = static_cast<double*>(ptebd::dev_alloc(&M, sizeof(double) * 256));
      M.ratio_bits = static_cast<unsigned long long*>(ptebd::dev_alloc(&M, sizeof(unsigned long long)));
      M.pwork = static_cast<double*>(ptebd::dev_alloc(&M, sizeof(double) * (5 * (size_t)sp + 8)));
    }
    const int64_t nbk = (r + 15) / 16 + 2;
    M.part_cap = (nbk / 2 + 1) * 16 * 1536;
    M.part = static_cast<double*>(ptebd::dev_alloc(&M, sizeof(double) * M.part_cap));
    M.info_i = static_cast<int*>(ptebd::dev_alloc(&M, sizeof(int) * 8));
    M.info_d = static_cast<double*>(ptebd::dev_alloc(&M, sizeof(double) * 16));
    M.counter = static_cast<unsigned int*>(ptebd::dev_alloc(&M, 64));
    M.ledger = static_cast<double*>(ptebd::dev_alloc(&M, 64));
    double* lam_out = static_cast<double*>(ptebd::dev_alloc(&M, sizeof(double) * r));
    PTEBD_HIP(hipHostMalloc((void**)&M.h_counter, 64, hipHostMallocDefault));
    PTEBD_HIP(hipHostMalloc((void**)&M.h_info, 64, hipHostMallocDefault));
    PTEBD_HIP(hipHostMalloc((void**)&M.h_part, 256 * sizeof(double), hipHostMallocDefault));
    PTEBD_HIP(hipHostMalloc((void**)&M.h_ratio, sizeof(unsigned long long), hipHostMallocDefault));
    PTEBD_HIP(hipMemcpy(a.re, A, sizeof(double) * m * n, hipMemcpyHostToDevice));
    PTEBD_HIP(hipMemcpy(a.im, A + (int64_t)m * n, sizeof(double) * m * n, hipMemcpyHostToDevice));
    PTEBD_HIP(hipMemset(M.ledger, 0, sizeof(double)));
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
    ptebd::mps_release(&M);
    (void)hipStreamDestroy(M.stream);
    return TEBD_OK;
  } catch (const ptebd::Error& e) {
    ptebd::set_last_error(e.what());
    ptebd::mps_release(&M);
    if (M.stream) (void)hipStreamDestroy(M.stream);
    return (tebd_status)e.code;
  }
}

extern "C" tebd_status tebd_diag_zgemm_time(int32_t prec, int32_t m, int32_t n, int32_t k, int32_t reps, double* ms) {
  if (m < 1 || n < 1 || k < 1 || reps < 1 || !ms || prec < 0 || prec > 2) return TEBD_EINVAL;
  try {
    Scratch sc;
    const int64_t na = (int64_t)m * k, nb = (int64_t)k * n, nc = (int64_t)m * n;
    double* a = sc.alloc(2 * na);
    double* b = sc.alloc(2 * nb);
    double* c = sc.alloc(2 * nc);
    ptebd::fill_random(a, 2 * na, 0x1234ull, nullptr);
    ptebd::fill_random(b, 2 * nb, 0x5678ull, nullptr);
    ptebd::ZGemmArgs g;
    g.m = m; g.n = n; g.k = k;
    g.ar = a; g.ai = a + na; g.lda = k;
    g.br = b; g.bi = b + nb; g.ldb = n;
    g.cr = c; g.ci = c + nc; g.ldc = n;
    ptebd::zgemm(g, prec, nullptr);
    hipEvent_t e0, e1;
    PTEBD_HIP(hipEventCreate(&e0));
    PTEBD_HIP(hipEventCreate(&e1));
    PTEBD_HIP(hipEventRecord(e0, nullptr));
    for (int i = 0; i < reps; ++i) ptebd::zgemm(g, prec, nullptr);
    PTEBD_HIP(hipEventRecord(e1, nullptr));
    PTEBD_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    PTEBD_HIP(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / reps;
    return TEBD_OK;
  } catch (const ptebd::Error& e) {
    ptebd::set_last_error(e.what());
    return (tebd_status)e.code;
  }
}

extern "C" tebd_status tebd_diag_gate(const tebd_model* m, int32_t supersite, int32_t j, double tau, double* G) {
  if (!m || !G || (supersite != 0 && supersite != 1) || !std::isfinite(tau)) return TEBD_EINVAL;
  if (m->L < 3 || m->d < 2 || m->d > 8 || !std::isfinite(m->U) || !std::isfinite(m->J) ||
      !std::isfinite(m->Jnnn) || !std::isfinite(m->K) || !std::isfinite(m->jc))
    return TEBD_EINVAL;
  if (supersite ? (m->L % 2 != 0 || m->L < 4 || j < 0 || j + 1 >= m->L / 2) : (j < 0 || j + 2 >= m->L))
    return TEBD_EINVAL;
  try {
    const ptebd::ModelP mp{m->L, m->d, m->U, m->J, m->Jnnn, m->K, m->jc};
    const ptebd::SpectralGate g = supersite ? ptebd::eig_supersite(mp, j) : ptebd::eig_three_site(mp, j);
    std::vector<double> re, im;
    ptebd::gate_matrix(g, tau, re, im);
    std::memcpy(G, re.data(), sizeof(double) * re.size());
    std::memcpy(G + re.size(), im.data(), sizeof(double) * im.size());
    return TEBD_OK;
  } catch (const ptebd::Error& e) {
    ptebd::set_last_error(e.what());
    return (tebd_status)e.code;
  } catch (const std::bad_alloc&) {
    ptebd::set_last_error("host allocation failed");
    return TEBD_ENOMEM;
  }
}

extern "C" tebd_status tebd_diag_bond_charges(int32_t L, int32_t d, const int32_t* chi, const double* B,
                                              int32_t* q) {
  if (L < 1 || d < 2 || d > 8 || !chi || !B || !q) return TEBD_EINVAL;
  if (chi[0] != 1 || chi[L] != 1) return TEBD_EINVAL;
  for (int b = 0; b <= L; ++b)
    if (chi[b] < 1) return TEBD_EINVAL;
  try {
    tebd_mps M;   // host fields only: no device memory is touched
    M.L = L;
    M.d = d;
    M.qs.resize(d);
    for (int t = 0; t < d; ++t) M.qs[t] = t;
    const std::vector<std::vector<int>> Q = ptebd::infer_charges(&M, chi, B);
    int64_t o = 0;
    for (const auto& qb : Q)
      for (int v : qb) q[o++] = v;
    return TEBD_OK;
  } catch (const ptebd::Error& e) {
    ptebd::set_last_error(e.what());
    return (tebd_status)e.code;
  } catch (const std::bad_alloc&) {
    ptebd::set_last_error("host allocation failed");
    return TEBD_ENOMEM;
  }
}
