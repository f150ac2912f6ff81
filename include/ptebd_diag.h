/*
 * ptebd_diag.h -- diagnostic entry points of the TEBD library.
 *
 * They run one building block of the gate update on device copies of host
 * arrays, so that tests can check each kernel in isolation against the CPU
 * oracle's primitives.  Host pointers in and out; the call allocates and
 * frees its own device memory and synchronises before returning.  Complex
 * arrays are planar (all real parts, then all imaginary parts), row-major.
 * Errors are reported as in ptebd.h.
 */
#ifndef PTEBD_DIAG_H
#define PTEBD_DIAG_H

#include "ptebd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C (m x n) = op(A) diag(k_scale) op(B), scaled by row_scale[i] * col_scale[j].
 * op(A) is A (stored m x k, leading dimension k) when transA == 0, or the
 * conjugate transpose of A stored k x m (leading dimension m) when transA == 1;
 * op(B) likewise (stored k x n, or n x k).  k_scale[k], row_scale[m],
 * col_scale[n] may be NULL.  prec is a tebd_precision.  herm != 0 declares
 * the product Hermitian (m == n, op(B) = op(A)^+, row_scale == col_scale):
 * only the lower tiles are computed and mirrored, as for Gram matrices. */
tebd_status tebd_diag_zgemm(int32_t prec, int32_t m, int32_t n, int32_t k, int32_t transA, int32_t transB,
                            const double* A, const double* B, const double* k_scale, const double* row_scale,
                            const double* col_scale, int32_t herm, double* C);

/* Truncated SVD of A (m x n) with the library's Jacobi engine and the
 * truncation rule of ptebd.h.  variant is a tebd_svd; the Gram routes need
 * eps >= TEBD_GRAM_EPS_MIN (else TEBD_EINVAL).  A single SVD has no warm
 * start, so TEBD_SVD_RANDOMIZED computes what TEBD_SVD_GRAM_EIG does.
 * Outputs: *k kept
 * values, s[0..k) the kept singular values renormalised to unit 2-norm,
 * vh (planar, k x n) the kept right singular vectors as rows, *nrm the
 * 2-norm of the kept values before renormalisation, *w the relative
 * discarded weight, *sweeps the Jacobi sweeps used.  s and vh must hold
 * min(m, n) and min(m, n) * n values (times two for vh). */
tebd_status tebd_diag_svd(int32_t variant, int32_t m, int32_t n, const double* A, int32_t chi_max, double w_max,
                          double eps, int32_t* k, double* s, double* vh, double* nrm, double* w, int32_t* sweeps);

/* tebd_diag_svd for callers that cannot allocate device memory (code that
 * must not call hipMalloc, tight serving loops, harnesses that forbid it):
 * the same computation, arguments and outputs, but every device buffer
 * (the input copy, the Jacobi and Gram workspaces, counters, the kept
 * vectors) is carved from one file-scope device array of 8 MiB that each
 * GPU holds until the process ends; the call makes no hipMalloc, hipFree or
 * host-pinned allocation.  Limits: m, n <= 512 and m * n <= 65536, else
 * TEBD_EINVAL before any device call.  Runs on the calling thread's current
 * device and its null stream, and synchronises before returning.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (from
 * several threads) race and must be serialised by the caller. */
tebd_status tebd_diag_svd_noalloc(int32_t variant, int32_t m, int32_t n, const double* A, int32_t chi_max,
                                  double w_max, double eps, int32_t* k, double* s, double* vh, double* nrm,
                                  double* w, int32_t* sweeps);

/* Per-call-site totals of the complex GEMM launches recorded by the handle's
 * profiler (mps_profile) since it was enabled: one text line per site,
 * "site launches device_ms algorithmic_flops", into out[cap] (NUL
 * terminated; EINVAL if it does not fit).  Synchronises. */
tebd_status tebd_diag_profile_sites(tebd_mps* mps, char* out, int64_t cap);

/* The process-wide tile tuner of the theta and gate products (FP64, shared
 * by every handle): counts[0] = (device, m, n, k, batch) shapes timed so far
 * (each with both the 64 x 64 and the 128 x 128 tile, three launches apiece,
 * the faster kept), counts[1] and counts[2] = later launches that took the
 * 64 x 64 and the 128 x 128 tile.  The environment variable
 * PTEBD_NO_AUTOTUNE switches the tuner off (the fixed launch rule then picks
 * every tile).  Host only. */
tebd_status tebd_diag_tile_tuner(int64_t* counts);

/* Average device time (ms, HIP events) of `reps` launches of the complex GEMM
 * kernel on device-resident m x k and k x n operands (contents unspecified,
 * finite), C = A B. */
tebd_status tebd_diag_zgemm_time(int32_t prec, int32_t m, int32_t n, int32_t k, int32_t reps, double* ms);

/* The gate G = exp(-i h tau) as the library builds it on the host in FP64
 * (Eq. (1) split into three-site terms h_j, or with supersite = 1 into the
 * two-super-site terms of super sites (j, j + 1), each diagonalised and
 * exponentiated).  Host only: no device call is made.  G (planar, n x n
 * row-major, output index first) must hold 2 n^2 values, n = d^3, or d^4 for
 * super sites.  EINVAL for an invalid model, j outside 0..L-3 (0..L/2-2 on
 * the super-site chain of even L >= 4) or a non-finite tau. */
tebd_status tebd_diag_gate(const tebd_model* m, int32_t supersite, int32_t j, double tau, double* G);

/* Particle number of every bond index (bosons to the left of the bond) as
 * mps_init_state infers it with tebd_opts.u1 on a three-site chain of L
 * sites of dimension d: chi[L + 1] bond dimensions (chi[0] = chi[L] = 1) and
 * the tensors B in mps_init_state's layout.  q receives chi[0] + ... + chi[L]
 * integers, bond by bond.  Host only: no device call is made.  EINVAL when an
 * index is reached by non-zero entries of two particle numbers or by none. */
tebd_status tebd_diag_bond_charges(int32_t L, int32_t d, const int32_t* chi, const double* B, int32_t* q);

#ifdef __cplusplus
}
#endif

#endif /* PTEBD_DIAG_H */
