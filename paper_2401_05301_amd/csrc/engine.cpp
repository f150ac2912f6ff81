// MPS store and the three-site gate update, driven from the host.
//
// Per gate on sites (j, j+1, j+2), with chi_l = chi_j, chi_r = chi_{j+3}:
//   T1   = B_j B_{j+1}                       (chi_l d) x (d chi_{j+2})      GEMM
//   psi  = T1 B_{j+2}                        (chi_l d^2) x (d chi_r)        GEMM
//   psi' = G psi  (batched over chi_l)       d^3 x chi_r per left index     GEMM
//   SVD #1 of M1 = Lambda_j psi' as (chi_l d) x (d^2 chi_r), truncate -> k1
//   B_j  = psi' V1 / |S1|                                                  GEMM
//   SVD #2 of M2 = S1 V1^+ as (k1 d) x (d chi_r), truncate -> k2
//   B_{j+2} = V2^+,  B_{j+1} = V1^+ V2 / |S2|                              GEMM
// The inverse-free form never divides by a Schmidt value.
#include "engine.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <functional>
#include <string>
#include <thread>

namespace ptebd {

namespace {

constexpr int kNsplitMax = 16;
// Gram route: singular values below this (relative) sit at the Gram
// matrix's rounding level; the subspace iteration does not chase them.
constexpr double kGramSigmaFloor = TEBD_GRAM_EPS_MIN;
constexpr double kDampRel = 1e-10;         // subspace iteration: power-step scale floor (relative to the top value)
constexpr double kDiagCoupling = 0.05;     // subspace iteration: largest relative coupling treated as diagonal
// Subspace iteration: largest Newton-Schulz scale (about the largest
// eigenvalue of the warm rows' normalised Gram matrix), or largest relative
// coupling of that Gram matrix, at which the warm rows are used as the start.
constexpr double kWarmMaxScale = 2.0;
constexpr double kWarmMaxCoupling = 0.5;
// Jacobi sweep limit when opts.max_sweeps <= 0.  Cyclic Jacobi on a matrix
// whose leading vectors are spread over many coordinates (raw-basis Gram
// blocks of a particle-number sector) can spend 30-40 sweeps in its linear
// phase before the quadratic one.
constexpr int kDefaultSweeps = 80;
// Gram matrices with fewer rows are solved directly (the subspace iteration
// pays only above about this size).
constexpr int kSubspaceMinRows = 1024;

int64_t ipow_cap(int d, int e, int cap) {
  int64_t v = 1;
  for (int i = 0; i < e; ++i) {
    v *= d;
    if (v >= cap) return cap;
  }
  return std::min<int64_t>(v, cap);
}

}  // namespace

void* dev_alloc(tebd_mps* M, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) / 256 * 256;
  void* p = nullptr;
  if (M->opts.dev_alloc) {
    p = M->opts.dev_alloc(bytes, M->opts.alloc_ctx);
    if (!p) throw Error(-2, "device allocation failed (allocator hook)");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(-2, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
  }
  M->allocs.push_back(p);
  return p;
}

namespace {

double* dalloc(tebd_mps* M, int64_t n) { return static_cast<double*>(dev_alloc(M, sizeof(double) * std::max<int64_t>(n, 1))); }

tebd_mps::Z zalloc(tebd_mps* M, int64_t n) {
  tebd_mps::Z z;
  z.re = dalloc(M, n);
  z.im = dalloc(M, n);
  return z;
}

}  // namespace

int64_t fused_table_bytes(int L) {
  // one entry per gate of a layer, and room for the gates of several handles
  // stepped together (tebd_step_many); then the SVD descriptors and ranks
  return (int64_t)(sizeof(JacobiArgs) + 2 * sizeof(int64_t) + 2 * sizeof(int) + sizeof(double)) *
             std::max(L + 1, kFusedMax) +
         128 + (int64_t)kFusedMax * (sizeof(FusedSvdArgs) + 2 * sizeof(int));
}

size_t Sizes::bytes(int workers, bool u1, bool fuse) const {
  int64_t d = 0;
  d += 2 * site_elems + lam_elems + 2 * (2 * meas_sq + 2 * meas_rect) + gates + 64;
  int64_t w = 2 * (T1 + 2 * psi + X2 + G + W + V1h);
  w += 2 * (4 * sub_p * sub_r + 6 * sub_p * sub_p);
  w += 6 * vec + part + 64 + 5 * sub_p + 8;
  if (u1) {
    w += 2 * uv + (idx + 4 * vec) / 2 + 1 + 2 * vec * (int64_t)(sizeof(RowCopy) / sizeof(double));
    // batched Jacobi tables
    w += ((int64_t)(std::max(sizeof(HermArgs), sizeof(JacobiArgs)) + 2 * sizeof(int64_t) + 2 * sizeof(int) +
                    sizeof(double)) * (vec / 2 + 1) + 128 + 7) / 8;
  } else if (fuse) {
    w += (fused_table_bytes((int)cap.size() - 1) + 7) / 8;
  }
  d += (int64_t)std::max(workers, 1) * w;
  return (size_t)d * sizeof(double);
}

int gates_per_layer(int L, bool super) { return super ? L / 2 : (L - 2 + 2) / 3; }

int auto_workers(int L, int requested, bool super, bool u1, bool fuse) {
  const int per_layer = std::max(1, gates_per_layer(L, super));
  // dense: six workers measured fastest on the bulk chi = 1024 chain (24.1 s per step
  // against 26.0 s with four and 24.6 s with eight); the latency-bound sector solves of
  // the U(1) route ran 27% slower with six than with four; a fused layer batches one
  // gate per workspace, so it takes one for every gate of a layer
  const int w = requested > 0 ? requested : fuse ? per_layer : (u1 ? 4 : 6);
  return std::max(1, std::min(w, per_layer));
}

int subspace_width(int r, int chi_max) {
  const int keep = std::min(chi_max, r);
  return std::max(subspace_width_keep(r, keep, false), subspace_width_keep(r, keep, true));
}

int subspace_width_keep(int r, int keep, bool wide) {
  // Oversampling: the narrow basis has keep / den extra rows, at least omin (den from
  // PTEBD_OVERSAMPLE_DEN, omin from PTEBD_OVERSAMPLE_MIN); the wide one keep / 4, at least 64.
  // The iteration contracts by lambda_{p+1} / lambda_k per step, so more rows mean fewer
  // iterations, but every iteration and every Jacobi sweep of its Rayleigh-Ritz grows with p.
  // On the bulk chi = 1024 workload the narrow basis is the faster one once the evolution
  // is under way, while the first gates after a canonicalisation converge only with the
  // wide one: the narrow basis runs first with a short iteration cap and the wide one
  // takes over when it has not converged.
  static const int den = std::getenv("PTEBD_OVERSAMPLE_DEN") ? std::max(1, std::atoi(std::getenv("PTEBD_OVERSAMPLE_DEN"))) : 16;
  static const int omin = std::getenv("PTEBD_OVERSAMPLE_MIN") ? std::max(1, std::atoi(std::getenv("PTEBD_OVERSAMPLE_MIN"))) : 64;
  const int extra = wide ? std::max(64, keep / 4) : std::max(omin, keep / den);
  const int p = ((keep + extra) + 15) / 16 * 16;
  // below ~1.5 p, or below kSubspaceMinRows rows, the whole Gram matrix is
  // cheaper to diagonalise directly (measured on the quench workload)
  return (3 * p < 2 * r && r >= kSubspaceMinRows) ? p : 0;
}

Sizes plan_sizes(int L, int d, int chi_max) {
  Sizes s;
  s.cap.resize(L + 1);
  for (int b = 0; b <= L; ++b) s.cap[b] = (int)ipow_cap(d, std::min(b, L - b), chi_max);
  const auto& c = s.cap;
  for (int i = 0; i < L; ++i) s.site_elems += (int64_t)c[i] * d * c[i + 1];
  for (int b = 0; b <= L; ++b) s.lam_elems += c[b];
  int64_t maxr = 1;
  for (int j = 0; j + 2 < L; ++j) {
    const int64_t cl = c[j], c2 = c[j + 2], cr = c[j + 3];
    const int64_t m1 = cl * d, n1 = (int64_t)d * d * cr, r1 = std::min(m1, n1);
    const int64_t k1 = std::min<int64_t>(r1, c[j + 1]);
    const int64_t m2 = k1 * d, n2 = (int64_t)d * cr, r2 = std::min(m2, n2);
    s.T1 = std::max(s.T1, cl * d * d * c2);
    s.psi = std::max(s.psi, cl * d * d * d * cr);
    s.V1h = std::max(s.V1h, k1 * n1);
    s.X2 = std::max(s.X2, m2 * n2);
    const int64_t k2 = std::min<int64_t>(r2, c2);
    s.uv = std::max(s.uv, std::max(k1 * n1, k2 * n2));
    s.idx = std::max(s.idx, std::max(m1 + n1, m2 + n2));
    s.G = std::max(s.G, std::max(r1 * r1, r2 * r2));
    s.vec = std::max(s.vec, std::max(std::max(r1, r2), std::max(m1, m2)));
    maxr = std::max(maxr, std::max(r1, r2));
    for (int64_t r : {r1, r2}) {
      const int64_t p = subspace_width((int)r, chi_max);
      if (p > 0) {
        s.sub_p = std::max(s.sub_p, p);
        s.sub_r = std::max(s.sub_r, r);
      }
    }
  }
  s.W = s.G;
  int chi = *std::max_element(c.begin(), c.end());
  s.meas_sq = (int64_t)chi * chi;
  s.meas_rect = (int64_t)chi * d * chi;
  s.vec = std::max<int64_t>(s.vec, (int64_t)chi * d);
  const int64_t nb = (maxr + 15) / 16 + 2;
  s.part = (nb / 2 + 1) * kNsplitMax * 1536;
  s.gates = (int64_t)std::max(L - 2, 0) * kGateSlots * 2 * (int64_t)d * d * d * d * d * d;
  return s;
}

Sizes plan_sizes2(int Ls, int D, int chi_max) {
  Sizes s;
  s.cap.resize(Ls + 1);
  for (int b = 0; b <= Ls; ++b) s.cap[b] = (int)ipow_cap(D, std::min(b, Ls - b), chi_max);
  const auto& c = s.cap;
  for (int i = 0; i < Ls; ++i) s.site_elems += (int64_t)c[i] * D * c[i + 1];
  for (int b = 0; b <= Ls; ++b) s.lam_elems += c[b];
  int64_t maxr = 1;
  s.T1 = 1;
  s.X2 = 1;
  s.V1h = 1;
  for (int K = 0; K + 1 < Ls; ++K) {
    const int64_t cl = c[K], cr = c[K + 2];
    const int64_t m = cl * D, n = (int64_t)D * cr, r = std::min(m, n);
    s.psi = std::max(s.psi, cl * D * D * cr);
    s.uv = std::max(s.uv, std::min<int64_t>(r, c[K + 1]) * n);
    s.idx = std::max(s.idx, m + n);
    s.G = std::max(s.G, r * r);
    s.vec = std::max(s.vec, std::max(m, n));
    maxr = std::max(maxr, r);
    const int64_t p = subspace_width((int)r, chi_max);
    if (p > 0) {
      s.sub_p = std::max(s.sub_p, p);
      s.sub_r = std::max(s.sub_r, r);
    }
  }
  s.W = s.G;
  const int chi = *std::max_element(c.begin(), c.end());
  s.meas_sq = (int64_t)chi * chi;
  s.meas_rect = (int64_t)chi * D * chi;
  s.vec = std::max<int64_t>(s.vec, (int64_t)chi * D);
  const int64_t nb = (maxr + 15) / 16 + 2;
  s.part = (nb / 2 + 1) * kNsplitMax * 1536;
  s.gates = (int64_t)std::max(Ls - 1, 0) * kGateSlots * 2 * (int64_t)D * D * D * D;
  return s;
}

namespace {

// Gate workspace of one worker W (sizes from plan_sizes).
void allocate_work(tebd_mps* W, const Sizes& s) {
  W->T1 = zalloc(W, s.T1);
  W->psi = zalloc(W, s.psi);
  W->psip = zalloc(W, s.psi);
  W->X2 = zalloc(W, s.X2);
  W->G = zalloc(W, s.G);
  W->g_cap = s.G;
  W->W = zalloc(W, s.W);
  W->V1h = zalloc(W, s.V1h);
  W->ks = dalloc(W, s.vec);
  W->norms = dalloc(W, s.vec);
  W->inv_sig = dalloc(W, s.vec);
  W->sq = dalloc(W, s.vec);
  W->perm = static_cast<int*>(dev_alloc(W, sizeof(int) * s.vec));
  W->flags = static_cast<int*>(dev_alloc(W, sizeof(int) * s.vec));
  W->flags_cap = s.vec;
  if (s.sub_p > 0 && W->opts.svd != TEBD_SVD_JACOBI) {
    const int64_t sp = s.sub_p;
    W->sub_p = (int)sp;
    W->sub_r = (int)s.sub_r;
    W->sZ = zalloc(W, sp * s.sub_r);
    W->sY = zalloc(W, sp * s.sub_r);
    W->sZ2 = zalloc(W, sp * s.sub_r);
    W->sY2 = zalloc(W, sp * s.sub_r);
    W->sH = zalloc(W, sp * sp);
    W->sW = zalloc(W, sp * sp);
    W->nY = zalloc(W, sp * sp);
    W->nZ = zalloc(W, sp * sp);
    W->nY2 = zalloc(W, sp * sp);
    W->nZ2 = zalloc(W, sp * sp);
    W->ns_part = dalloc(W, 256);
    W->ratio_bits = static_cast<unsigned long long*>(dev_alloc(W, sizeof(unsigned long long)));
    W->pwork = dalloc(W, 5 * sp + 8);
  }
  W->part = dalloc(W, s.part);
  W->part_cap = s.part;
  if (W->opts.u1) {
    W->u_idx_cap = s.idx + 4 * s.vec;
    W->u_idx = static_cast<int*>(dev_alloc(W, sizeof(int) * W->u_idx_cap));
    W->u_tab_cap = 2 * s.vec;
    W->u_tab = static_cast<RowCopy*>(dev_alloc(W, sizeof(RowCopy) * W->u_tab_cap));
    W->uv = zalloc(W, s.uv);
    // at most one batched matrix per two values of the union (each has n >= 2)
    const int64_t cnt = s.vec / 2 + 1;
    W->u_batch_cap =
        (int64_t)(std::max(sizeof(HermArgs), sizeof(JacobiArgs)) + 2 * sizeof(int64_t) + 2 * sizeof(int) +
                  sizeof(double)) * cnt + 128;
    W->u_batch = dev_alloc(W, (size_t)W->u_batch_cap);
  } else if (W->opts.fuse) {
    // batched Jacobi tables of a fused layer, then the SVD descriptors
    W->u_batch_cap = (int64_t)(sizeof(JacobiArgs) + 2 * sizeof(int64_t) + 2 * sizeof(int) + sizeof(double)) *
                         std::max(W->L + 1, kFusedMax) +
                     128;
    W->u_batch = dev_alloc(W, (size_t)W->u_batch_cap);
    W->f_tab = static_cast<FusedSvdArgs*>(dev_alloc(W, sizeof(FusedSvdArgs) * kFusedMax));
    W->f_k = static_cast<int*>(dev_alloc(W, sizeof(int) * 2 * kFusedMax));
    PTEBD_HIP(hipHostMalloc((void**)&W->h_ftab, sizeof(FusedSvdArgs) * kFusedMax, hipHostMallocDefault));
    PTEBD_HIP(hipHostMalloc((void**)&W->h_fk, sizeof(int) * 2 * kFusedMax, hipHostMallocDefault));
  }
  W->info_i = static_cast<int*>(dev_alloc(W, sizeof(int) * 8));
  W->info_d = dalloc(W, 16);
  W->counter = static_cast<unsigned int*>(dev_alloc(W, sizeof(unsigned int) * 4));
  PTEBD_HIP(hipHostMalloc((void**)&W->h_counter, 64, hipHostMallocDefault));
  PTEBD_HIP(hipHostMalloc((void**)&W->h_info, 64, hipHostMallocDefault));
  PTEBD_HIP(hipHostMalloc((void**)&W->h_part, 256 * sizeof(double), hipHostMallocDefault));
  PTEBD_HIP(hipHostMalloc((void**)&W->h_ratio, sizeof(unsigned long long), hipHostMallocDefault));
}

}  // namespace

void mps_allocate(tebd_mps* M) {
  Sizes s = M->super ? plan_sizes2(M->L, M->d, M->chi_max) : plan_sizes(M->L, M->d, M->chi_max);
  M->cap = s.cap;
  M->chi.assign(M->L + 1, 1);
  const int L = M->L, d = M->d;
  M->Br.resize(L);
  M->Bi.resize(L);
  for (int i = 0; i < L; ++i) {
    const int64_t n = (int64_t)M->cap[i] * d * M->cap[i + 1];
    M->Br[i] = dalloc(M, n);
    M->Bi[i] = dalloc(M, n);
  }
  M->lam.resize(L + 1);
  for (int b = 0; b <= L; ++b) M->lam[b] = dalloc(M, M->cap[b]);
  M->ledger = dalloc(M, 1);
  M->wslots = dalloc(M, L);
  M->E = zalloc(M, s.meas_sq);
  M->F2 = zalloc(M, s.meas_sq);
  M->F = zalloc(M, s.meas_rect);
  M->F3 = zalloc(M, s.meas_rect);
  M->ks = dalloc(M, s.vec);
  M->meas = dalloc(M, 8 * (int64_t)std::max(L, M->phys_L) + 8);
  M->hop_part = dalloc(M, 512);
  M->d_br = static_cast<double**>(dev_alloc(M, sizeof(double*) * L));
  M->d_bi = static_cast<double**>(dev_alloc(M, sizeof(double*) * L));
  M->d_lam = static_cast<double**>(dev_alloc(M, sizeof(double*) * (L + 1)));
  M->d_chi = static_cast<int*>(dev_alloc(M, sizeof(int) * (L + 1)));
  PTEBD_HIP(hipMemcpyAsync(M->d_br, M->Br.data(), sizeof(double*) * L, hipMemcpyHostToDevice, M->stream));
  PTEBD_HIP(hipMemcpyAsync(M->d_bi, M->Bi.data(), sizeof(double*) * L, hipMemcpyHostToDevice, M->stream));
  PTEBD_HIP(hipMemcpyAsync(M->d_lam, M->lam.data(), sizeof(double*) * (L + 1), hipMemcpyHostToDevice, M->stream));
  fill_zero(M->ledger, 1, M->stream);
  const int nw = auto_workers(L, M->opts.workers, M->super, M->opts.u1 != 0, M->opts.fuse != 0);
  for (int w = 0; w < nw; ++w) {
    tebd_mps* W = new tebd_mps();
    M->workers.push_back(W);
    W->parent = M;
    W->opts = M->opts;
    W->L = M->L;
    W->d = M->d;
    W->chi_max = M->chi_max;
    if (w == 0) {
      W->stream = M->stream;
    } else {
      PTEBD_HIP(hipStreamCreateWithFlags(&W->stream, hipStreamNonBlocking));
      W->own_stream = true;
    }
    allocate_work(W, s);
  }
  PTEBD_HIP(hipStreamSynchronize(M->stream));
}

void mps_release(tebd_mps* M) {
  for (tebd_mps* W : M->workers) {
    mps_release(W);
    if (W->own_stream) (void)hipStreamDestroy(W->stream);
    delete W;
  }
  M->workers.clear();
  if (M->stream) (void)hipStreamSynchronize(M->stream);
  for (void* p : M->allocs) {
    if (M->opts.dev_free)
      M->opts.dev_free(p, M->opts.alloc_ctx);
    else
      (void)hipFree(p);
  }
  M->allocs.clear();
  if (M->h_counter) (void)hipHostFree(M->h_counter);
  if (M->h_info) (void)hipHostFree(M->h_info);
  if (M->h_part) (void)hipHostFree(M->h_part);
  if (M->h_ratio) (void)hipHostFree(M->h_ratio);
  if (M->h_ftab) (void)hipHostFree(M->h_ftab);
  if (M->h_fk) (void)hipHostFree(M->h_fk);
  M->h_ftab = nullptr;
  M->h_fk = nullptr;
  M->h_ratio = nullptr;
  M->h_counter = nullptr;
  M->h_info = nullptr;
  M->h_part = nullptr;
}

void upload_product(tebd_mps* M, const int* occ) {
  if (M->super) {
    // super site K holds physical sites 2K, 2K+1 as the index s_{2K} d + s_{2K+1}
    std::vector<int> so(M->L);
    for (int K = 0; K < M->L; ++K) so[K] = occ[2 * K] * M->pd + occ[2 * K + 1];
    const int L = M->L, d = M->d;
    std::vector<double> zr(d), zi(d, 0.0);
    for (int i = 0; i < L; ++i) {
      std::fill(zr.begin(), zr.end(), 0.0);
      zr[so[i]] = 1.0;
      PTEBD_HIP(hipMemcpy(M->Br[i], zr.data(), sizeof(double) * d, hipMemcpyHostToDevice));
      PTEBD_HIP(hipMemcpy(M->Bi[i], zi.data(), sizeof(double) * d, hipMemcpyHostToDevice));
    }
    const double one = 1.0;
    for (int b = 0; b <= L; ++b) PTEBD_HIP(hipMemcpy(M->lam[b], &one, sizeof(double), hipMemcpyHostToDevice));
    M->chi.assign(L + 1, 1);
    M->q.assign(L + 1, std::vector<int>(1, 0));
    for (int b = 1; b <= L; ++b) M->q[b][0] = M->q[b - 1][0] + M->qs[so[b - 1]];
    return;
  }
  const int L = M->L, d = M->d;
  std::vector<double> zr(d), zi(d, 0.0);
  for (int i = 0; i < L; ++i) {
    std::fill(zr.begin(), zr.end(), 0.0);
    zr[occ[i]] = 1.0;
    PTEBD_HIP(hipMemcpy(M->Br[i], zr.data(), sizeof(double) * d, hipMemcpyHostToDevice));
    PTEBD_HIP(hipMemcpy(M->Bi[i], zi.data(), sizeof(double) * d, hipMemcpyHostToDevice));
  }
  const double one = 1.0;
  for (int b = 0; b <= L; ++b) PTEBD_HIP(hipMemcpy(M->lam[b], &one, sizeof(double), hipMemcpyHostToDevice));
  M->chi.assign(L + 1, 1);
  M->q.assign(L + 1, std::vector<int>(1, 0));
  for (int b = 1; b <= L; ++b) M->q[b][0] = M->q[b - 1][0] + M->qs[occ[b - 1]];
}

void upload_state(tebd_mps* M, const int* chi, const double* B, const double* lam) {
  const int L = M->L, d = M->d;
  if (M->u1) M->q = infer_charges(M, chi, B);
  int64_t off = 0;
  for (int i = 0; i < L; ++i) {
    const int64_t n = (int64_t)chi[i] * d * chi[i + 1];
    PTEBD_HIP(hipMemcpy(M->Br[i], B + off, sizeof(double) * n, hipMemcpyHostToDevice));
    PTEBD_HIP(hipMemcpy(M->Bi[i], B + off + n, sizeof(double) * n, hipMemcpyHostToDevice));
    off += 2 * n;
  }
  off = 0;
  for (int b = 0; b <= L; ++b) {
    PTEBD_HIP(hipMemcpy(M->lam[b], lam + off, sizeof(double) * chi[b], hipMemcpyHostToDevice));
    off += chi[b];
  }
  M->chi.assign(chi, chi + L + 1);
}

void set_model(tebd_mps* M, const ModelP& m) {
  M->model = m;
  M->spectra.clear();
  if (M->super)
    for (int K = 0; K + 1 < M->L; ++K) M->spectra.push_back(eig_supersite(m, K));
  else
    for (int j = 0; j + 2 < M->L; ++j) M->spectra.push_back(eig_three_site(m, j));
  // device gates are rebuilt lazily into the same buffers (the caller has
  // synchronised the handle, so no launch still reads them)
  M->gates.resize(M->spectra.size());
  for (auto& slots : M->gates) {
    slots.resize(kGateSlots);
    for (auto& g : slots) g.valid = false;
  }
}

namespace {

// G_j(tau) on the device: a resident slot of window j if one holds this tau,
// else the least recently used slot is rebuilt (allocated on first use; a
// slot that held another gate is overwritten only after the handle's stream
// has drained, so no launch still reads it).
std::pair<double*, double*> device_gate(tebd_mps* M, int j, double tau) {
  auto& slots = M->gates[j];
  tebd_mps::GateSlot* pick = nullptr;
  for (auto& g : slots)
    if (g.valid && g.tau == tau) {
      g.used = ++M->gate_clock;
      return {g.re, g.im};
    }
  for (auto& g : slots)
    if (!pick || (!g.valid && pick->valid) || (g.valid == pick->valid && g.used < pick->used)) pick = &g;
  std::vector<double> re, im;
  gate_matrix(M->spectra[j], tau, re, im);
  if (!pick->re) {
    pick->re = dalloc(M, (int64_t)re.size());
    pick->im = dalloc(M, (int64_t)im.size());
  } else if (pick->valid) {
    PTEBD_HIP(hipStreamSynchronize(M->stream));
  }
  PTEBD_HIP(hipMemcpy(pick->re, re.data(), sizeof(double) * re.size(), hipMemcpyHostToDevice));
  PTEBD_HIP(hipMemcpy(pick->im, im.data(), sizeof(double) * im.size(), hipMemcpyHostToDevice));
  pick->tau = tau;
  pick->valid = true;
  pick->used = ++M->gate_clock;
  return {pick->re, pick->im};
}

bool debug_enabled() {
  static const bool on = std::getenv("PTEBD_DEBUG") != nullptr;
  return on;
}

// Launch shape of the one-sided Jacobi on the r rows (length c) of X, with
// the rotations accumulated into W when wr is set: 16-row blocks, column
// splits of the pair Grams, column chunks of the update.
JacobiArgs jacobi_args(double* xr, double* xi, int64_t ldx, double* wr, double* wi, int64_t ldw, int r, int c,
                       double tol_rel, double tol_abs) {
  int nb = (r + 15) / 16;
  if (nb < 2) nb = 2;
  if (nb & 1) ++nb;
  const int npairs = nb / 2;
  JacobiArgs a{};
  a.xr = xr; a.xi = xi; a.ldx = ldx;
  a.wr = wr; a.wi = wi; a.ldw = ldw;
  a.r = r; a.c = c; a.nb = nb;
  a.nsplit = std::max(1, std::min({kNsplitMax, (c + 63) / 64, (1024 + npairs - 1) / npairs}));
  const int total = c + (wr ? r : 0);
  int nu = std::max(1, std::min((total + 63) / 64, (1024 + npairs - 1) / npairs));
  a.ucols = ((total + nu - 1) / nu + 15) / 16 * 16;
  a.nuchunks = (total + a.ucols - 1) / a.ucols;
  a.tol_rel = tol_rel;
  a.tol_abs = tol_abs;
  return a;
}

int64_t jacobi_part(const JacobiArgs& a) { return (int64_t)(a.nb / 2) * a.nsplit * 1536; }

// One-sided block Jacobi on the rows of X; returns the number of sweeps.
int run_jacobi(tebd_mps* M, double* xr, double* xi, int64_t ldx, double* wr, double* wi, int64_t ldw, int r, int c,
               double tol_rel, double tol_abs) {
  hipStream_t s = M->stream;
  JacobiArgs a = jacobi_args(xr, xi, ldx, wr, wi, ldw, r, c, tol_rel, tol_abs);
  const int nb = a.nb;
  if (jacobi_part(a) > M->part_cap) throw Error(-1, "Jacobi scratch too small");
  a.part = M->part;
  a.rotated = M->counter;
  row_norms(xr, xi, ldx, r, c, M->norms, s);
  negligible_norm2(M->norms, r, M->info_d + 6, s);
  a.tiny2 = M->info_d + 6;
  {
    // Rows left at the rounding level by the rotations of a rank-deficient
    // X carry noise of order u |X|_F, and so do their inner products: an
    // inner product below (64 u |X|_F)^2 counts as converged, whatever the
    // norms of the two rows (tiny2 = (4 u)^2 |X|_F^2).
    double t2 = 0.0;
    PTEBD_HIP(hipMemcpyAsync(&t2, M->info_d + 6, sizeof(double), hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipStreamSynchronize(s));
    a.tol_abs = std::max(a.tol_abs, 256.0 * t2);
  }
  if (wr) set_identity(wr, wi, ldw, r, s);
  if (const char* dump = std::getenv("PTEBD_DUMP")) {
    // debugging aid: keep the last Jacobi input on disk (r, c, then planar data)
    std::vector<double> h(2 * (size_t)r * c);
    PTEBD_HIP(hipMemcpy2DAsync(h.data(), sizeof(double) * c, xr, sizeof(double) * ldx, sizeof(double) * c, r,
                               hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipMemcpy2DAsync(h.data() + (size_t)r * c, sizeof(double) * c, xi, sizeof(double) * ldx,
                               sizeof(double) * c, r, hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipStreamSynchronize(s));
    if (FILE* f = std::fopen(dump, "wb")) {
      const int32_t dims[2] = {r, c};
      std::fwrite(dims, sizeof(int32_t), 2, f);
      std::fwrite(h.data(), sizeof(double), h.size(), f);
      std::fclose(f);
    }
  }
  const int max_sweeps = M->opts.max_sweeps > 0 ? M->opts.max_sweeps : kDefaultSweeps;
  for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
    fill_zero_words(M->counter, 1, s);
    for (int t = 0; t < nb - 1; ++t) jacobi_round(a, t, s);
    PTEBD_HIP(hipMemcpyAsync(M->h_counter, M->counter, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipStreamSynchronize(s));
    if (debug_enabled())
      std::fprintf(stderr, "[ptebd] jacobi r=%d c=%d W=%d sweep=%d rotated_pairs=%u\n", r, c, wr != nullptr, sweep,
                   *M->h_counter);
    if (*M->h_counter == 0) {
      M->last_sweeps = sweep;
      M->total_sweeps += sweep;
      return sweep;
    }
  }
  M->failed = true;
  throw Error(-4, "Jacobi SVD did not converge within max_sweeps (rows " + std::to_string(r) + ", columns " +
                      std::to_string(c) + ")");
}

// run_jacobi on a group of independent matrices at once (each JacobiArgs
// with its own part scratch): every round launches the pair Grams and the
// rotations of all matrices still rotating, so that small matrices share the
// device instead of running their latency-bound rounds one after the other.
// Every matrix takes the launch shape, tolerances and sweeps it would take
// alone, so its result is the same bit for bit.
void run_jacobi_group(tebd_mps* M, std::vector<JacobiArgs>& tab,
                      const std::function<void(double* tiny2)>& prologue = nullptr) {
  hipStream_t s = M->stream;
  const int count = (int)tab.size();
  // device layout in u_batch: JacobiArgs[count], gram_first[count+1], rot_first[count+1],
  // active[count], counts[count], tiny2[count]
  const size_t need = sizeof(JacobiArgs) * count + 2 * sizeof(int64_t) * (count + 1) + 2 * sizeof(int) * count +
                      sizeof(double) * count + 64;
  if ((int64_t)need > M->u_batch_cap) throw Error(-1, "batched Jacobi tables exceed their buffer");
  char* base = static_cast<char*>(M->u_batch);
  JacobiArgs* d_tab = reinterpret_cast<JacobiArgs*>(base);
  int64_t* d_gram = reinterpret_cast<int64_t*>(d_tab + count);
  int64_t* d_rot = d_gram + (count + 1);
  int* d_active = reinterpret_cast<int*>(d_rot + (count + 1));
  unsigned int* d_counts = reinterpret_cast<unsigned int*>(d_active + count);
  double* d_tiny2 = reinterpret_cast<double*>(reinterpret_cast<char*>(d_counts + count) +
                                              ((8 - (reinterpret_cast<uintptr_t>(d_counts + count) & 7)) & 7));
  std::vector<int64_t>& first = M->h_first;
  first.assign(2 * (count + 1), 0);
  int max_nb = 0;
  // the floor of every matrix into d_tiny2[i] and the identity into its
  // vectors: one matrix after the other, or in one batch by the caller
  if (prologue) prologue(d_tiny2);
  for (int i = 0; i < count; ++i) {
    JacobiArgs& a = tab[i];
    if (!prologue) {
      row_norms(a.xr, a.xi, a.ldx, a.r, a.c, M->norms, s);
      negligible_norm2(M->norms, a.r, d_tiny2 + i, s);
      if (a.wr) set_identity(a.wr, a.wi, a.ldw, a.r, s);
    }
    a.tiny2 = d_tiny2 + i;
    a.rotated = d_counts + i;
    first[i + 1] = first[i] + (int64_t)(a.nb / 2) * a.nsplit;
    first[count + 1 + i + 1] = first[count + 1 + i] + (int64_t)(a.nb / 2) * a.nuchunks;
    max_nb = std::max(max_nb, a.nb);
  }
  {
    // the absolute floor of run_jacobi, per matrix
    std::vector<double> t2(count);
    PTEBD_HIP(hipMemcpyAsync(t2.data(), d_tiny2, sizeof(double) * count, hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < count; ++i) tab[i].tol_abs = std::max(tab[i].tol_abs, 256.0 * t2[i]);
  }
  PTEBD_HIP(hipMemcpyAsync(d_tab, tab.data(), sizeof(JacobiArgs) * count, hipMemcpyHostToDevice, s));
  PTEBD_HIP(hipMemcpyAsync(d_gram, first.data(), sizeof(int64_t) * 2 * (count + 1), hipMemcpyHostToDevice, s));
  std::vector<int>& act = M->h_active;
  act.assign(count, 1);
  std::vector<unsigned int>& cnt = M->h_counts;
  cnt.assign(count, 0);
  const int max_sweeps = M->opts.max_sweeps > 0 ? M->opts.max_sweeps : kDefaultSweeps;
  int rounds = max_nb - 1;
  for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
    PTEBD_HIP(hipMemcpyAsync(d_active, act.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    fill_zero_words(d_counts, count, s);
    for (int t = 0; t < rounds; ++t)
      jacobi_round_batched(d_tab, d_gram, first[count], d_rot, first[2 * (count + 1) - 1], count, d_active, t, s);
    PTEBD_HIP(hipMemcpyAsync(cnt.data(), d_counts, sizeof(unsigned int) * count, hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipStreamSynchronize(s));
    rounds = 0;
    for (int i = 0; i < count; ++i) {
      if (act[i] && cnt[i] == 0) act[i] = 0;
      if (act[i]) rounds = std::max(rounds, tab[i].nb - 1);
    }
    if (debug_enabled()) {
      std::string line;
      for (int i = 0; i < count; ++i)
        if (act[i]) line += " " + std::to_string(tab[i].r) + "x" + std::to_string(tab[i].c) + ":" +
                            std::to_string(cnt[i]);
      std::fprintf(stderr, "[ptebd] batched one-sided jacobi sweep=%d rotating(r x c:pairs)%s\n", sweep,
                   line.c_str());
    }
    if (rounds == 0) {
      M->last_sweeps = sweep;
      M->total_sweeps += sweep;
      return;
    }
  }
  M->failed = true;
  throw Error(-4, "batched Jacobi SVD did not converge within max_sweeps (" + std::to_string(count) + " matrices)");
}

// run_jacobi on every matrix of tab, in groups whose pair Grams fit the
// scratch together.
void run_jacobi_batched(tebd_mps* M, std::vector<JacobiArgs>& tab) {
  size_t i0 = 0;
  while (i0 < tab.size()) {
    std::vector<JacobiArgs> group;
    int64_t poff = 0;
    size_t i1 = i0;
    while (i1 < tab.size()) {
      const int64_t need = jacobi_part(tab[i1]);
      if (need > M->part_cap) throw Error(-1, "Jacobi scratch too small");
      if (poff + need > M->part_cap) break;
      group.push_back(tab[i1]);
      group.back().part = M->part + poff;
      poff += need;
      ++i1;
    }
    run_jacobi_group(M, group);
    i0 = i1;
  }
}

// Truncated SVD of diag(rs) A.  Writes the kept normalised singular values
// into lam_out, V^+ rows into (vhr, vhi) with leading dimension n, the norm of
// the kept values into info_d[2*slot] and returns k.
// Off-diagonal target of the Hermitian Jacobi in units of u trace(H).  The
// entries of a Gram matrix M M^+ carry absolute errors of order
// u sqrt(k) |m_i| |m_j| themselves; an unresolved off-diagonal entry delta
// leaves the Schmidt basis off diagonal by delta, an error of that size in
// the local observables.
double herm_tol_units() {
  static const double v = std::getenv("PTEBD_HERM_TOL") ? std::atof(std::getenv("PTEBD_HERM_TOL")) : 64.0;
  return v;
}

// Jacobi sweeps of an intermediate rotation of the subspace iteration.
int partial_sweeps() {
  static const int v = std::getenv("PTEBD_PARTIAL_SWEEPS") ? std::atoi(std::getenv("PTEBD_PARTIAL_SWEEPS")) : 4;
  return v;
}

// Subspace iteration stopping tolerance: largest residual of a kept basis
// row relative to the trace of the Gram matrix (the squared norm of theta).
// A kept Schmidt vector weighted by its value is off by about that much,
// so 1e-12 keeps the observables well inside the 1e-10 FP64 bar.
double sub_res_rel() {
  static const double v = std::getenv("PTEBD_SUB_RES") ? std::atof(std::getenv("PTEBD_SUB_RES")) : 1e-12;
  return v;
}

int inner_sweeps() {
  static const int v = std::getenv("PTEBD_INNER_SWEEPS") ? std::atoi(std::getenv("PTEBD_INNER_SWEEPS")) : 1;
  return v;
}

// Two-sided block Jacobi on the Hermitian H (n x n) in place, eigenvector rows
// accumulated into W (set to the identity first).  Returns the sweeps used.
// With sweep_cap > 0 at most that many sweeps run and an unconverged H is
// returned as it stands (partial diagonalisation), without an error.
// The off-diagonal target is c u trace(H); with a trace_of block given
// (the whole matrix, of which H is a diagonal block) the target is taken
// against its trace instead, so that a block of rounding noise is not
// chased below the rounding level of the whole.
int run_herm_jacobi(tebd_mps* M, double* hr, double* hi, int64_t ldh, int n, double* wr, double* wi, int64_t ldw,
                    int sweep_cap = 0, const double* trace_of = nullptr, int trace_n = 0) {
  hipStream_t s = M->stream;
  int nb = (n + 15) / 16;
  if (nb < 2) nb = 2;
  if (nb & 1) ++nb;
  const int npairs = nb / 2;
  if ((int64_t)npairs * 2048 > M->part_cap) throw Error(-1, "Hermitian Jacobi scratch too small");
  HermArgs a{};
  a.hr = hr; a.hi = hi; a.ldh = ldh; a.n = n; a.nb = nb;
  a.wr = wr; a.wi = wi; a.ldw = ldw;
  a.wcols = 128;
  a.wchunks = (n + a.wcols - 1) / a.wcols;
  a.qbuf = M->part;
  a.flag = M->flags;
  a.inner_sweeps = inner_sweeps();
  a.rotated = M->counter;
  if (trace_of)
    herm_tol(trace_of, ldh, trace_n, herm_tol_units(), M->info_d + 7, s);
  else
    herm_tol(hr, ldh, n, herm_tol_units(), M->info_d + 7, s);
  a.tol_abs = M->info_d + 7;
  if (wr) set_identity(wr, wi, ldw, n, s);
  const int max_sweeps = sweep_cap > 0 ? sweep_cap : (M->opts.max_sweeps > 0 ? M->opts.max_sweeps : kDefaultSweeps);
  if (debug_enabled()) std::fprintf(stderr, "[ptebd] herm-jacobi start n=%d cap=%d\n", n, sweep_cap);
  // Convergence is checked before every sweep by counting the off-diagonal
  // entries above the target, so no sweep runs only to find nothing to do.
  auto converged = [&]() {
    const unsigned above = count_above(hr, hi, ldh, n, a.tol_abs, M->counter + 1, M->h_counter + 1, s);
    return above == 0;
  };
  for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
    if (converged()) {
      M->last_sweeps = sweep - 1;
      M->total_sweeps += sweep - 1;
      return sweep - 1;
    }
    fill_zero_words(M->counter, 1, s);
    for (int t = 0; t < nb - 1; ++t) herm_round(a, t, s);
    if (debug_enabled()) {
      PTEBD_HIP(hipMemcpyAsync(M->h_counter, M->counter, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
      PTEBD_HIP(hipStreamSynchronize(s));
      std::fprintf(stderr, "[ptebd] herm-jacobi n=%d sweep=%d rotated_pairs=%u\n", n, sweep, *M->h_counter);
    }
  }
  if (sweep_cap > 0) {
    M->last_sweeps = sweep_cap;
    M->total_sweeps += sweep_cap;
    return sweep_cap;
  }
  if (converged()) {
    M->last_sweeps = max_sweeps;
    M->total_sweeps += max_sweeps;
    return max_sweeps;
  }
  M->failed = true;
  throw Error(-4, "Hermitian Jacobi did not converge within max_sweeps (n " + std::to_string(n) + ")");
}

// Symmetric (Loewdin) orthonormalisation of the rows of Z (p x r): rows are
// normalised, then Z <- (Z Z^+)^{-1/2} Z.  Of all orthonormal bases of the row
// space this one is closest to Z, so a basis that was already nearly
// orthonormal (Ritz vectors and their images) keeps its alignment.  The
// inverse square root of A = Z Z^+ comes from the coupled Newton-Schulz
// iteration Y <- Y T, X <- T X, T = (3 I - X Y) / 2 started from Y = A / c,
// X = I, with c >= lambda_max(A) (Gershgorin), so that X -> (A / c)^{-1/2}.
// With in_place the result is copied back into Z's memory (Z may then be a
// view of leading rows of a larger basis); otherwise Z and T swap.
// With soft set, a Newton-Schulz run that does not converge returns false
// (Z unchanged, the handle left usable) instead of failing the handle.
// With max_c > 0 the call gives up (returns false) before iterating when
// the scale c exceeds max_c, i.e. when the normalised rows are too far from
// orthonormal for the iteration to converge quickly.
bool lowdin(tebd_mps* M, tebd_mps::Z& Z, tebd_mps::Z& T, int p, int r, bool in_place = false, bool soft = false,
            double max_c = 0.0) {
  hipStream_t s = M->stream;
  normalize_rows(Z.re, Z.im, r, p, r, nullptr, s);
  // every product below is a polynomial in the Hermitian A, hence Hermitian:
  // only the lower-triangular tiles are computed
  auto mm = [&](const tebd_mps::Z& A, const tebd_mps::Z& B, tebd_mps::Z& C) {
    ZGemmArgs g;
    g.m = p; g.n = p; g.k = p;
    g.ar = A.re; g.ai = A.im; g.lda = p;
    g.br = B.re; g.bi = B.im; g.ldb = p;
    g.cr = C.re; g.ci = C.im; g.ldc = p;
    g.herm_out = 1;
    g.tag = "ns_product";
    zgemm(g, 0, s);
  };
  {
    ZGemmArgs g;
    g.m = p; g.n = p; g.k = r;
    g.ar = Z.re; g.ai = Z.im; g.lda = r;
    g.br = Z.re; g.bi = Z.im; g.ldb = r; g.transB = 1;
    g.cr = M->sH.re; g.ci = M->sH.im; g.ldc = p;
    g.herm_out = 1;
    g.tag = "lowdin_gram";
    zgemm(g, 0, s);
  }
  double* c = M->info_d + 8;   // c, sqrt(c)
  // The scale c must exceed lambda_max(A) (the iteration converges for
  // eigenvalues of A / c in (0, 3)); the closer it is, the fewer iterations.
  // A power-iteration estimate times 1.3 is used, capped by the Gershgorin
  // bound; a diverging run restarts from the Gershgorin bound alone.
  bool safe = false;
  ns_scale(M->sH.re, M->sH.im, p, M->pwork, 12, 1.3, c, s);
  if (max_c > 0.0) {
    double hc = 0.0;
    PTEBD_HIP(hipMemcpyAsync(&hc, c, sizeof(double), hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipStreamSynchronize(s));
    if (!(hc <= max_c)) {
      if (debug_enabled()) std::fprintf(stderr, "[ptebd] lowdin p=%d: rows too far from orthonormal (c=%.3f)\n", p, hc);
      return false;
    }
  }
  ns_init(M->sH.re, M->sH.im, p, c, M->nY.re, M->nY.im, M->nZ.re, M->nZ.im, s);
  const double tol2 = 1e-28 * p;
  int it = 0;
  double prev_dev = 0.0;
  for (; it < 40; ++it) {
    mm(M->nZ, M->nY, M->sW);                       // P = X Y
    const int g = ns_three_minus(M->sW.re, M->sW.im, p, M->ns_part, s);   // T = (3I - P)/2
    mm(M->nY, M->sW, M->nY2);                      // Y <- Y T
    mm(M->sW, M->nZ, M->nZ2);                      // X <- T X
    std::swap(M->nY, M->nY2);
    std::swap(M->nZ, M->nZ2);
    PTEBD_HIP(hipMemcpyAsync(M->h_part, M->ns_part, sizeof(double) * g, hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipStreamSynchronize(s));
    double dev = 0.0;
    for (int b = 0; b < g; ++b) dev += M->h_part[b];
    if (dev <= tol2) break;
    if (!safe && (!(dev < 1e300) || (it >= 3 && dev > 4.0 * prev_dev))) {
      safe = true;
      ns_scale(M->sH.re, M->sH.im, p, M->pwork, 0, 0.0, c, s);
      ns_init(M->sH.re, M->sH.im, p, c, M->nY.re, M->nY.im, M->nZ.re, M->nZ.im, s);
      dev = 0.0;
    }
    prev_dev = dev;
  }
  if (debug_enabled()) {
    double hc = 0.0;
    PTEBD_HIP(hipMemcpyAsync(&hc, c, sizeof(double), hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipStreamSynchronize(s));
    std::fprintf(stderr, "[ptebd] lowdin p=%d newton-schulz iterations=%d c=%.3f\n", p, it + 1, hc);
  }
  if (it == 40) {
    if (soft) return false;
    M->failed = true;
    throw Error(-4, "Newton-Schulz orthonormalisation did not converge (basis of width " + std::to_string(p) + ")");
  }
  // Z <- A^{-1/2} Z = X Z / sqrt(c)
  ZGemmArgs q;
  q.m = p; q.n = r; q.k = p;
  q.ar = M->nZ.re; q.ai = M->nZ.im; q.lda = p;
  q.br = Z.re; q.bi = Z.im; q.ldb = r;
  q.cr = T.re; q.ci = T.im; q.ldc = r;
  q.alpha_dev = c + 1; q.alpha_recip = 1;
  q.tag = "lowdin_apply";
  zgemm(q, 0, s);
  if (in_place) {
    PTEBD_HIP(hipMemcpyAsync(Z.re, T.re, sizeof(double) * (size_t)p * r, hipMemcpyDeviceToDevice, s));
    PTEBD_HIP(hipMemcpyAsync(Z.im, T.im, sizeof(double) * (size_t)p * r, hipMemcpyDeviceToDevice, s));
  } else {
    std::swap(Z, T);
  }
  return true;
}

// Orthonormalisation of the subspace basis: Cholesky-QR unless
// PTEBD_LOWDIN selects the symmetric Newton-Schulz route (tuning switch).
bool lowdin_selected() {
  static const bool v = std::getenv("PTEBD_LOWDIN") != nullptr;
  return v;
}

// Hermitian C = A B^+ (p x p, leading dimension p) for row blocks A and B of
// p rows of length r (leading dimension r).  With K = r long against the few
// tiles of C (p ~ 1100 gives 153 work-groups of 64 x 64), the product is
// split into ns slices of K computed as one batched launch into the scratch
// (ns p^2 values per plane) and summed slice by slice in a fixed order, so
// that the result does not depend on timing.
void herm_product_split(tebd_mps* M, const double* ar, const double* ai, const double* br, const double* bi, int p,
                        int r, double* cr, double* ci, tebd_mps::Z scratch, int64_t scratch_elems, const char* tag) {
  hipStream_t s = M->stream;
  const int64_t tiles = (int64_t)ceil_div(p, 64) * (ceil_div(p, 64) + 1) / 2;
  int ns = (int)std::min<int64_t>(8, std::max<int64_t>(1, (600 + tiles - 1) / tiles));
  ns = (int)std::min<int64_t>(ns, scratch_elems / ((int64_t)p * p));
  ns = std::min(ns, r / 256);   // slices of at least 256
  ZGemmArgs g;
  g.m = p; g.n = p;
  g.ar = ar; g.ai = ai; g.lda = r;
  g.br = br; g.bi = bi; g.ldb = r; g.transB = 1;
  g.herm_out = 1;
  g.tag = tag;
  if (ns <= 1) {
    g.k = r;
    g.cr = cr; g.ci = ci; g.ldc = p;
    zgemm(g, 0, s);
    return;
  }
  // slices of ceil(r / ns) rounded up to a multiple of 16, the last one shorter:
  // at most ns slices in all
  const int slice = ((r + ns - 1) / ns + 15) / 16 * 16;
  const int nf = r / slice, rest = r - nf * slice;
  g.k = slice; g.batch = nf;
  g.sA = slice; g.sB = slice; g.sC = (int64_t)p * p;
  g.cr = scratch.re; g.ci = scratch.im; g.ldc = p;
  zgemm(g, 0, s);
  int total = nf;
  if (rest > 0) {
    ZGemmArgs t = g;
    t.k = rest; t.batch = 1; t.sA = t.sB = t.sC = 0;
    t.ar = ar + (int64_t)nf * slice; t.ai = ai + (int64_t)nf * slice;
    t.br = br + (int64_t)nf * slice; t.bi = bi + (int64_t)nf * slice;
    t.cr = scratch.re + (int64_t)nf * p * p; t.ci = scratch.im + (int64_t)nf * p * p;
    zgemm(t, 0, s);
    ++total;
  }
  sum_slices(scratch.re, scratch.im, (int64_t)p * p, total, cr, ci, s);
}

// Orthonormal rows by Cholesky-QR (Gram-Schmidt in row order): the rows of
// Z (p x r) are normalised, K = Z Z^+ = L L^+ is factorised and Z <- L^-1 Z.
// Row i changes only by its components along rows 0..i-1, so a basis that is
// nearly orthonormal barely moves, and the work is two GEMM-shaped products
// (K and the application of L^-1) plus a small blocked factorisation.  With
// max_coupling > 0 the call gives up (returns false) when some
// |K_ij| / sqrt(K_ii K_jj) exceeds it: rows that far from orthogonal are not
// worth keeping as a start.  It also returns false if the factorisation
// breaks down (dependent rows).  Uses sH, nY and nZ as scratch; the result
// replaces Z (swapped with T, or copied into Z's memory when in_place).
bool orthonormalize(tebd_mps* M, tebd_mps::Z& Z, tebd_mps::Z& T, int p, int r, bool in_place,
                    double max_coupling = 0.0) {
  if (lowdin_selected()) return lowdin(M, Z, T, p, r, in_place, true, max_coupling > 0.0 ? kWarmMaxScale : 0.0);
  hipStream_t s = M->stream;
  normalize_rows(Z.re, Z.im, r, p, r, nullptr, s);
  // K = Z Z^+ (T is free until the final product and holds the slices)
  herm_product_split(M, Z.re, Z.im, Z.re, Z.im, p, r, M->sH.re, M->sH.im, T, (int64_t)M->sub_p * M->sub_r,
                     "ortho_gram");
  if (max_coupling > 0.0) {
    herm_tol(M->sH.re, p, p, herm_tol_units(), M->info_d + 7, s);
    const double ratio = offdiag_ratio(M->sH.re, M->sH.im, p, p, M->info_d + 7, 0.0, M->ratio_bits, M->h_ratio, s);
    if (!(ratio <= max_coupling)) {
      if (debug_enabled()) std::fprintf(stderr, "[ptebd] cholesky-qr p=%d: rows far from orthogonal (%.2e)\n", p, ratio);
      return false;
    }
  }
  int* flag = M->info_i + 6;
  fill_zero_words(flag, 1, s);
  chol_inverse(M->sH.re, M->sH.im, p, M->nY.re, M->nY.im, M->nZ.re, M->nZ.im, flag, s);
  PTEBD_HIP(hipMemcpyAsync(M->h_info + 6, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  PTEBD_HIP(hipStreamSynchronize(s));
  if (M->h_info[6]) {
    if (debug_enabled()) std::fprintf(stderr, "[ptebd] cholesky-qr p=%d: factorisation broke down\n", p);
    return false;
  }
  {
    ZGemmArgs q;
    q.m = p; q.n = r; q.k = p;
    q.ar = M->nY.re; q.ai = M->nY.im; q.lda = p;
    q.br = Z.re; q.bi = Z.im; q.ldb = r;
    q.cr = T.re; q.ci = T.im; q.ldc = r;
    q.tag = "ortho_apply";
    zgemm(q, 0, s);
  }
  if (in_place) {
    PTEBD_HIP(hipMemcpyAsync(Z.re, T.re, sizeof(double) * (size_t)p * r, hipMemcpyDeviceToDevice, s));
    PTEBD_HIP(hipMemcpyAsync(Z.im, T.im, sizeof(double) * (size_t)p * r, hipMemcpyDeviceToDevice, s));
  } else {
    std::swap(Z, T);
  }
  return true;
}

// H = Y Z^+ (p x p) for the basis rows Z and their images Y = Z G (Hermitian:
// Z G Z^+).  sY2 is free here and holds the slices.
void rayleigh(tebd_mps* M, int p, int r) {
  herm_product_split(M, M->sY.re, M->sY.im, M->sZ.re, M->sZ.im, p, r, M->sH.re, M->sH.im, M->sY2,
                     (int64_t)M->sub_p * M->sub_r, "rayleigh");
}

// Independent Hermitian matrices (H n x n in place, eigenvector rows into W,
// both with leading dimension n) for one batched Jacobi.
struct BatchItem {
  double* hr;
  double* hi;
  double* wr;
  double* wi;
  int n;
};

// Two-sided block Jacobi on every matrix of the batch at once: each round
// launches the pair solves and the rotations of all matrices still above
// the threshold (c u times the summed trace of the batch), so small
// matrices share the device instead of running their latency-bound rounds
// one after the other.  Convergence is counted per matrix before every
// sweep.
void run_herm_jacobi_batched(tebd_mps* M, const std::vector<BatchItem>& items) {
  hipStream_t s = M->stream;
  const int count = (int)items.size();
  // device layout in u_batch: HermArgs[count], eig_first[count+1], app_first[count+1],
  // active[count], counts[count], tol[count]
  const size_t need = sizeof(HermArgs) * count + 2 * sizeof(int64_t) * (count + 1) + 2 * sizeof(int) * count +
                      sizeof(double) * count + 64;
  if ((int64_t)need > M->u_batch_cap) throw Error(-1, "batched Jacobi tables exceed their buffer");
  char* base = static_cast<char*>(M->u_batch);
  HermArgs* d_tab = reinterpret_cast<HermArgs*>(base);
  int64_t* d_eig = reinterpret_cast<int64_t*>(d_tab + count);
  int64_t* d_app = d_eig + (count + 1);
  int* d_active = reinterpret_cast<int*>(d_app + (count + 1));
  unsigned int* d_counts = reinterpret_cast<unsigned int*>(d_active + count);
  double* d_tol = reinterpret_cast<double*>(reinterpret_cast<char*>(d_counts + count) +
                                            ((8 - (reinterpret_cast<uintptr_t>(d_counts + count) & 7)) & 7));
  std::vector<HermArgs>& tab = M->h_herm;
  tab.assign(count, HermArgs{});
  std::vector<int64_t>& first = M->h_first;
  first.assign(2 * (count + 1), 0);
  int64_t qoff = 0, foff = 0;
  int max_n = 0;
  for (int i = 0; i < count; ++i) {
    const BatchItem& it = items[i];
    HermArgs& a = tab[i];
    int nb = (it.n + 15) / 16;
    if (nb < 2) nb = 2;
    if (nb & 1) ++nb;
    a.hr = it.hr; a.hi = it.hi; a.ldh = it.n; a.n = it.n; a.nb = nb;
    a.wr = it.wr; a.wi = it.wi; a.ldw = it.n;
    a.wcols = 128;
    a.wchunks = (it.n + a.wcols - 1) / a.wcols;
    a.qbuf = M->part + qoff;
    a.flag = M->flags + foff;
    a.rotated = M->counter;
    a.tol_abs = d_tol + i;
    a.inner_sweeps = inner_sweeps();
    qoff += (int64_t)(nb / 2) * 2 * 32 * 32;
    foff += nb / 2;
    first[i + 1] = first[i] + nb / 2;
    first[count + 1 + i + 1] = first[count + 1 + i] + herm_apply_groups(a);
    max_n = std::max(max_n, it.n);
    herm_tol(it.hr, it.n, it.n, herm_tol_units(), d_tol + i, s);
    set_identity(it.wr, it.wi, it.n, it.n, s);
  }
  if (qoff > M->part_cap || foff > M->flags_cap) throw Error(-1, "U(1) SVD: batched Jacobi scratch too small");
  // The sector Gram matrices are diagonal blocks of one Gram matrix, whose
  // entries all carry absolute errors of order u times its trace: every
  // sector takes the threshold of the whole (the sum of the sector
  // thresholds), the target the dense route uses, instead of chasing
  // rounding noise below it in the small sectors.
  share_sum(d_tol, count, s);
  PTEBD_HIP(hipMemcpyAsync(d_tab, tab.data(), sizeof(HermArgs) * count, hipMemcpyHostToDevice, s));
  PTEBD_HIP(hipMemcpyAsync(d_eig, first.data(), sizeof(int64_t) * 2 * (count + 1), hipMemcpyHostToDevice, s));
  std::vector<int>& act = M->h_active;
  act.assign(count, 1);
  std::vector<unsigned int>& cnt = M->h_counts;
  cnt.assign(count, 0);
  const int max_sweeps = M->opts.max_sweeps > 0 ? M->opts.max_sweeps : kDefaultSweeps;
  PTEBD_HIP(hipMemcpyAsync(d_active, act.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
  for (int sweep = 0;; ++sweep) {
    fill_zero_words(d_counts, count, s);
    count_above_batched(d_tab, count, d_active, max_n, d_counts, s);
    PTEBD_HIP(hipMemcpyAsync(cnt.data(), d_counts, sizeof(unsigned int) * count, hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipStreamSynchronize(s));
    int rounds = 0;
    for (int i = 0; i < count; ++i) {
      if (act[i] && cnt[i] == 0) act[i] = 0;
      if (act[i]) rounds = std::max(rounds, tab[i].nb - 1);
    }
    if (debug_enabled()) {
      std::string line;
      for (int i = 0; i < count; ++i)
        if (act[i]) line += " " + std::to_string(tab[i].n) + ":" + std::to_string(cnt[i]);
      std::fprintf(stderr, "[ptebd] batched-jacobi sweep=%d active(n:above)%s\n", sweep, line.c_str());
    }
    if (rounds == 0) {
      M->last_sweeps = sweep;
      M->total_sweeps += sweep;
      return;
    }
    if (sweep == max_sweeps) {
      M->failed = true;
      throw Error(-4, "batched Hermitian Jacobi did not converge within max_sweeps (" + std::to_string(count) +
                          " sectors)");
    }
    PTEBD_HIP(hipMemcpyAsync(d_active, act.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    for (int t = 0; t < rounds; ++t)
      herm_round_batched(d_tab, d_eig, first[count], d_app, first[2 * (count + 1) - 1], count,
                         d_active, t, s);
  }
}

// Top-p eigenpairs of the Hermitian PSD G (r x r) by subspace iteration with
// Rayleigh-Ritz.  On return sZ holds the Ritz vectors as rows (conjugated,
// as W in run_herm_jacobi), M->norms the Ritz values, and info_d[5] the
// weight of G outside the subspace (trace minus the Ritz values).
// Returns false when the iteration breaks down (an orthonormalisation that
// does not converge, a Rayleigh matrix that is not positive semi-definite, or
// kept values still moving at the last iteration: a start nearly inside the
// null space of a rank-deficient G); the caller then solves G directly.
bool subspace_topk(tebd_mps* M, const double* gr, const double* gi, int r, int p, int keep, const WarmStart& w,
                   int max_it) {
  hipStream_t s = M->stream;
  fill_random(M->sZ.re, (int64_t)p * r, 0x5eed1234abcdull, s);
  fill_random(M->sZ.im, (int64_t)p * r, 0x0bad5eedfeedull, s);
  // eigenpairs of the Rayleigh matrix (partially with a sweep cap)
  auto rr_jacobi = [&](int cap) { run_herm_jacobi(M, M->sH.re, M->sH.im, p, p, M->sW.re, M->sW.im, p, cap); };
  int kw = 0;   // warm rows at the top of the basis
  if (w.kind == 1 && w.src_cols <= p && w.src_rows == r) {
    conj_transpose_scaled(w.sr, w.si, w.ld, w.rs, w.rdiv, w.src_rows, w.src_cols, M->sZ.re, M->sZ.im, r, s);
    kw = w.src_cols;
  } else if (w.kind == 2 && w.src_rows <= p && w.src_cols == r) {
    scale_rows_copy(w.sr, w.si, w.ld, nullptr, 1, w.src_rows, w.src_cols, M->sZ.re, M->sZ.im, r, s);
    kw = w.src_rows;
  }
  if (kw > 0 && kw < p) {
    // Orthonormalise the warm rows on their own and take the random rows
    // out of their span, so that the basis keeps the warm rows as they are
    // (a joint symmetric orthonormalisation would mix them with noise).
    // Warm rows of a state in canonical form are orthogonal already; rows
    // far from that (a state that is not canonical yet) give no useful
    // start, and the basis starts from random rows instead.
    if (!orthonormalize(M, M->sZ, M->sZ2, kw, r, true, kWarmMaxCoupling)) {
      kw = 0;
      fill_random(M->sZ.re, (int64_t)p * r, 0x5eed1234abcdull, s);
      fill_random(M->sZ.im, (int64_t)p * r, 0x0bad5eedfeedull, s);
    }
  }
  if (kw > 0 && kw < p) {
    tebd_mps::Z rnd{M->sZ.re + (size_t)kw * r, M->sZ.im + (size_t)kw * r};
    ZGemmArgs c;   // C = R Zw^+  ((p - kw) x kw)
    c.m = p - kw; c.n = kw; c.k = r;
    c.ar = rnd.re; c.ai = rnd.im; c.lda = r;
    c.br = M->sZ.re; c.bi = M->sZ.im; c.ldb = r; c.transB = 1;
    c.cr = M->sH.re; c.ci = M->sH.im; c.ldc = kw;
    c.tag = "warm_overlap";
    zgemm(c, 0, s);
    ZGemmArgs u;   // R <- R - C Zw
    u.m = p - kw; u.n = r; u.k = kw;
    u.ar = M->sH.re; u.ai = M->sH.im; u.lda = kw;
    u.br = M->sZ.re; u.bi = M->sZ.im; u.ldb = r;
    u.cr = rnd.re; u.ci = rnd.im; u.ldc = r;
    u.alpha = -1.0; u.beta = 1;
    u.tag = "warm_project";
    zgemm(u, 0, s);
    if (!orthonormalize(M, rnd, M->sZ2, p - kw, r, true)) return false;
  } else {
    if (!orthonormalize(M, M->sZ, M->sZ2, p, r, false)) return false;
    if (!orthonormalize(M, M->sZ, M->sZ2, p, r, false)) return false;
  }
  // trace of G: scale of the rounding noise in the Ritz values
  tail_rest(gr, r, r, M->norms, 0, M->info_d + 4, s);
  double trace = 0.0;
  PTEBD_HIP(hipMemcpyAsync(&trace, M->info_d + 4, sizeof(double), hipMemcpyDeviceToHost, s));
  PTEBD_HIP(hipStreamSynchronize(s));
  std::vector<double> h_res(p), sorted;
  auto image = [&]() {   // Y = Z G (rows: (G z_i)^+), H = Y Z^+
    ZGemmArgs g;
    g.m = p; g.n = r; g.k = r;
    g.ar = M->sZ.re; g.ai = M->sZ.im; g.lda = r;
    g.br = gr; g.bi = gi; g.ldb = r;
    g.cr = M->sY.re; g.ci = M->sY.im; g.ldc = r;
    g.tag = "subspace_image";
    zgemm(g, 0, s);
    rayleigh(M, p, r);
  };
  // rows [r0, r0 + n) of Z (and Y) <- Q rows [r0, r0 + n), Q (n x n, leading dimension n)
  auto rotate = [&](const tebd_mps::Z& Q, int r0, int n, bool also_y) {
    for (int t = 0; t < (also_y ? 2 : 1); ++t) {
      tebd_mps::Z& X = t == 0 ? M->sZ : M->sY;
      tebd_mps::Z& T = t == 0 ? M->sZ2 : M->sY2;
      ZGemmArgs q;
      q.m = n; q.n = r; q.k = n;
      q.ar = Q.re; q.ai = Q.im; q.lda = n;
      q.br = X.re + (size_t)r0 * r; q.bi = X.im + (size_t)r0 * r; q.ldb = r;
      q.cr = T.re + (size_t)r0 * r; q.ci = T.im + (size_t)r0 * r; q.ldc = r;
      q.tag = "subspace_rotate";
      zgemm(q, 0, s);
      if (r0 == 0 && n == p) {
        std::swap(X, T);
      } else {
        PTEBD_HIP(hipMemcpyAsync(X.re + (size_t)r0 * r, T.re + (size_t)r0 * r, sizeof(double) * (size_t)n * r,
                                 hipMemcpyDeviceToDevice, s));
        PTEBD_HIP(hipMemcpyAsync(X.im + (size_t)r0 * r, T.im + (size_t)r0 * r, sizeof(double) * (size_t)n * r,
                                 hipMemcpyDeviceToDevice, s));
      }
    }
  };
  std::vector<double> h_vals(p);
  for (int it = 0; it < max_it; ++it) {
    image();
    if (it == 0 && kw > 0 && kw < p) {
      // The random rows carry no structure: diagonalise their own block
      // first, so that H is nearly diagonal as a whole.
      const int nr = p - kw;
      run_herm_jacobi(M, M->sH.re + (size_t)kw * p + kw, M->sH.im + (size_t)kw * p + kw, p, nr, M->sW.re,
                      M->sW.im, nr, 0, M->sH.re, p);
      rotate(M->sW, kw, nr, true);
      rayleigh(M, p, r);
    }
    herm_diag(M->sH.re, p, p, M->norms, s);
    // Next basis.  The exact power step spans the rows of Z + H^-1 R with
    // the block residual R = Y - H Z (orthogonal to every basis row).  When
    // the couplings of H are small against its diagonal (relative to
    // sqrt(H_ii H_jj), with the damping floor), diag(H) stands in for H.
    // Otherwise a few Jacobi sweeps first rotate the basis towards the Ritz
    // vectors; they need not converge, since the residual is taken against
    // the rotated H as it stands.
    PTEBD_HIP(hipMemcpyAsync(h_vals.data(), M->norms, sizeof(double) * p, hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipStreamSynchronize(s));
    const double top0 = *std::max_element(h_vals.begin(), h_vals.end());
    herm_tol(M->sH.re, p, p, herm_tol_units(), M->info_d + 7, s);
    const double ratio = offdiag_ratio(M->sH.re, M->sH.im, p, p, M->info_d + 7, kDampRel * top0, M->ratio_bits,
                                       M->h_ratio, s);
    if (!(ratio <= 1.5)) {
      // |H_ij| <= sqrt(H_ii H_jj) holds for the positive semi-definite
      // Z G Z^+: a larger coupling means the basis has lost its accuracy
      if (debug_enabled()) std::fprintf(stderr, "[ptebd] subspace r=%d p=%d: Rayleigh matrix not PSD (%.2e)\n", r, p, ratio);
      return false;
    }
    const bool jac = !(ratio <= kDiagCoupling);
    if (jac) {
      rr_jacobi(partial_sweeps());
      herm_diag(M->sH.re, p, p, M->norms, s);
      rotate(M->sW, 0, p, true);
    }
    {  // Y <- Y - (H - diag(H)) Z: row i becomes theta_i z_i + R_i
      zero_diag(M->sH.re, M->sH.im, p, p, s);
      ZGemmArgs q;
      q.m = p; q.n = r; q.k = p;
      q.ar = M->sH.re; q.ai = M->sH.im; q.lda = p;
      q.br = M->sZ.re; q.bi = M->sZ.im; q.ldb = r;
      q.cr = M->sY.re; q.ci = M->sY.im; q.ldc = r;
      q.alpha = -1.0; q.beta = 1;
      q.tag = "subspace_residual";
      zgemm(q, 0, s);
    }
    // Stopping rule: the residual |R_i| = |G z_i - sum_j H_ij z_j| of every
    // basis row whose Rayleigh quotient is among the `keep` largest.  It
    // bounds the angle between the span and the eigenvectors it should hold
    // by |R| / gap, so once it is below tol * trace G every kept Schmidt
    // vector, weighted by its value, is off by at most about that much.
    residual_norms(M->sY.re, M->sY.im, M->sZ.re, M->sZ.im, r, p, r, M->norms, M->sq, s);
    PTEBD_HIP(hipMemcpyAsync(h_vals.data(), M->norms, sizeof(double) * p, hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipMemcpyAsync(h_res.data(), M->sq, sizeof(double) * p, hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipStreamSynchronize(s));
    sorted.assign(h_vals.begin(), h_vals.end());
    std::nth_element(sorted.begin(), sorted.begin() + (keep - 1), sorted.end(), std::greater<double>());
    const double kth = sorted[keep - 1];
    double top = 0.0, res = 0.0;
    for (int i = 0; i < p; ++i) {
      top = std::max(top, h_vals[i]);
      if (h_vals[i] >= kth) res = std::max(res, h_res[i]);
    }
    const bool done = it >= 1 && res <= sub_res_rel() * trace;
    if (debug_enabled())
      std::fprintf(stderr, "[ptebd] subspace r=%d p=%d it=%d residual=%.3e (of trace %.3e) kth=%.3e top=%.6e %s %.2e\n",
                   r, p, it, res, trace, kth, top, jac ? "jacobi" : "diag", ratio);
    if (done) {
      // final Rayleigh-Ritz: exact eigenvectors of H (its diagonal restored)
      set_diag(M->sH.re, M->sH.im, p, p, M->norms, s);
      rr_jacobi(0);
      herm_diag(M->sH.re, p, p, M->norms, s);
      rotate(M->sW, 0, p, false);
      break;
    }
    if (it == max_it - 1) {
      // the span has not settled on the leading eigenvectors (a start
      // nearly inside the null space of a rank-deficient G): the caller
      // solves G directly
      if (debug_enabled()) std::fprintf(stderr, "[ptebd] subspace r=%d p=%d: not converged\n", r, p);
      return false;
    }
    // Damped power step: a plain image G Z has rows spread over the whole
    // dynamic range of G and is too ill-conditioned to orthonormalise
    // accurately; scaling each image by its Ritz value and capping the
    // residual step keeps the rows near orthonormal.
    damped_power_rows(M->sZ.re, M->sZ.im, M->sY.re, M->sY.im, r, p, r, M->norms, 1.0, kDampRel,
                      kGramSigmaFloor * kGramSigmaFloor, s);
    std::swap(M->sZ, M->sY);
    if (!orthonormalize(M, M->sZ, M->sZ2, p, r, false)) {
      if (debug_enabled()) std::fprintf(stderr, "[ptebd] subspace r=%d p=%d: orthonormalisation failed\n", r, p);
      return false;
    }
  }
  tail_rest(gr, r, r, M->norms, p, M->info_d + 5, s);
  return true;
}

// Relative orthogonality target of the one-sided Jacobi for rows of length c:
// a few times the rounding error of a length-c dot product.
double jacobi_tol(int c) { return std::max(2e-15, 2.0 * std::sqrt((double)c) * 1.11e-16); }

// Smallest kept Schmidt value, relative to the largest, below which the rows
// V^+ = S^-1 U^+ M of the left Gram route are re-orthonormalised.  An
// eigenvector u_i of the Gram matrix carries a component of order
// u / s_j^2 along a larger u_j (u the unit roundoff), and the division by
// s_i turns it into a component of order u / (s_i s_j) of v_j in v_i: up to
// ~1e-10 next to s_j ~ 1 for s_i ~ 1e-6, enough to move the observables by
// the FP64 bar.  Cholesky-QR of the rows in order of decreasing value
// (Gram-Schmidt) removes exactly those components.
constexpr double kRefineRatio = 1e-3;

// Iteration caps of the subspace iteration: the narrow basis gives up early
// (the wide one converges where it does not), the wide one before the direct
// solve of the whole Gram matrix.
constexpr int kNarrowIters = 10;
constexpr int kWideIters = 30;

// Cholesky-QR of the k rows of V (length n, leading dimension ldv) in their
// stored order: V <- L^-1 V with V V^+ = L L^+, so that row i loses its
// components along rows 0..i-1 and every row ends with unit norm.  Uses the
// Gram and eigenvector workspaces (G, W) and out (k x n, n >= k) as scratch;
// leaves V unchanged if the factorisation breaks down (rows dependent).
void cholqr_rows(tebd_mps* M, double* vr, double* vi, int64_t ldv, int k, int n, tebd_mps::Z out) {
  hipStream_t s = M->stream;
  if (k < 2) return;
  if ((int64_t)k * k > M->g_cap) throw Error(-1, "Cholesky-QR: k^2 exceeds the Gram workspace");
  if (n < k) throw Error(-1, "Cholesky-QR: fewer columns than rows");
  {  // K = V V^+
    ZGemmArgs g;
    g.m = k; g.n = k; g.k = n;
    g.ar = vr; g.ai = vi; g.lda = ldv;
    g.br = vr; g.bi = vi; g.ldb = ldv; g.transB = 1;
    g.cr = M->G.re; g.ci = M->G.im; g.ldc = k;
    g.herm_out = 1;
    g.tag = "refine_gram";
    zgemm(g, 0, s);
  }
  int* flag = M->info_i + 6;
  fill_zero_words(flag, 1, s);
  chol_inverse(M->G.re, M->G.im, k, M->W.re, M->W.im, out.re, out.im, flag, s);
  PTEBD_HIP(hipMemcpyAsync(M->h_info + 6, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  PTEBD_HIP(hipStreamSynchronize(s));
  if (M->h_info[6]) {
    if (debug_enabled()) std::fprintf(stderr, "[ptebd] cholesky-qr k=%d: factorisation broke down, rows kept\n", k);
    return;
  }
  {  // out = L^-1 V
    ZGemmArgs q;
    q.m = k; q.n = n; q.k = k;
    q.ar = M->W.re; q.ai = M->W.im; q.lda = k;
    q.br = vr; q.bi = vi; q.ldb = ldv;
    q.cr = out.re; q.ci = out.im; q.ldc = n;
    q.tag = "refine_apply";
    zgemm(q, 0, s);
  }
  scale_rows_copy(out.re, out.im, n, nullptr, 1, k, n, vr, vi, ldv, s);
}

// Counts the part of the truncation rule that set the k just read back
// (h_info[4], written by select_truncate).
void count_rule(tebd_mps* M) {
  const int rule = M->h_info[4];
  if (rule >= 0 && rule < 4) ++M->rule_counts[rule];
}

}  // namespace

int svd_trunc(tebd_mps* M, const SvdIn& in, double* lam_out, double* vhr, double* vhi, int slot, tebd_mps::Z xbuf) {
  hipStream_t s = M->stream;
  const int m = in.m, n = in.n;
  const bool gram = M->opts.svd != TEBD_SVD_JACOBI;
  double* nrm = M->info_d + 2 * slot;
  int* kdev = M->info_i + slot;
  const double eps = M->opts.trunc_rel;
  const double w_max = M->opts.trunc_weight;
  if (!gram) {
    if (m <= n) {
      scale_rows_copy(in.ar, in.ai, in.lda, in.rs, in.rdiv, m, n, xbuf.re, xbuf.im, n, s);
      run_jacobi(M, xbuf.re, xbuf.im, n, nullptr, nullptr, 0, m, n, jacobi_tol(n),
                 0.0);
      row_norms(xbuf.re, xbuf.im, n, m, n, M->norms, s);
      select_truncate(M->norms, m, 0, M->chi_max, w_max, eps, lam_out, M->perm, M->inv_sig, kdev, nrm, M->ledger, nullptr, s);
      PTEBD_HIP(hipMemcpyAsync(M->h_info, kdev, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
      PTEBD_HIP(hipStreamSynchronize(s));
      const int k = M->h_info[0];
      count_rule(M);
      gather_rows(xbuf.re, xbuf.im, n, M->perm, M->inv_sig, k, n, vhr, vhi, n, kdev, s);
      return k;
    } else {
      conj_transpose_scaled(in.ar, in.ai, in.lda, in.rs, in.rdiv, m, n, xbuf.re, xbuf.im, m, s);
      run_jacobi(M, xbuf.re, xbuf.im, m, M->W.re, M->W.im, n, n, m, jacobi_tol(m),
                 0.0);
      row_norms(xbuf.re, xbuf.im, m, n, m, M->norms, s);
      select_truncate(M->norms, n, 0, M->chi_max, w_max, eps, lam_out, M->perm, M->inv_sig, kdev, nrm, M->ledger, nullptr, s);
      PTEBD_HIP(hipMemcpyAsync(M->h_info, kdev, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
      PTEBD_HIP(hipStreamSynchronize(s));
      const int k = M->h_info[0];
      count_rule(M);
      gather_rows(M->W.re, M->W.im, n, M->perm, nullptr, k, n, vhr, vhi, n, kdev, s);
      return k;
    }
  }
  // Gram route: G = A_s A_s^+ (m <= n) or A_s^+ A_s (m > n), r x r.  The
  // caller's eps is used as given: the handle refuses eps below
  // TEBD_GRAM_EPS_MIN on this route, so every cut of the rule lies well
  // above the Gram matrix's rounding level.
  const double eps_g = eps;
  // The smaller Gram matrix, except that the right one is kept where the
  // warm start lives on that side and the subspace iteration will run on
  // it, unless it is clearly the larger one (and while it fits the Gram
  // workspace).
  bool left = in.prefer_right ? (m < n) : (m <= n);
  if (in.prefer_right && left && 5 * (int64_t)m >= 4 * (int64_t)n && M->sub_p > 0 &&
      (int64_t)n * n <= M->g_cap) {
    const int pr = subspace_width(n, M->chi_max);
    if (pr > 0 && pr <= M->sub_p && n <= M->sub_r) left = false;
  }
  const int r = left ? m : n;
  if (left) {
    ZGemmArgs g;
    g.m = m; g.n = m; g.k = n;
    g.ar = in.ar; g.ai = in.ai; g.lda = in.lda;
    g.br = in.ar; g.bi = in.ai; g.ldb = in.lda; g.transB = 1;
    g.cr = M->G.re; g.ci = M->G.im; g.ldc = m;
    g.row_scale = in.rs; g.row_div = in.rdiv;
    g.col_scale = in.rs; g.col_div = in.rdiv;
    g.herm_out = 1;
    g.tag = "gram";
    zgemm(g, 0, s);
  } else {
    const double* ks = nullptr;
    if (in.rs) {
      square_expand(in.rs, in.rdiv, m, M->sq, s);
      ks = M->sq;
    }
    ZGemmArgs g;
    g.m = n; g.n = n; g.k = m;
    g.ar = in.ar; g.ai = in.ai; g.lda = in.lda; g.transA = 1;
    g.br = in.ar; g.bi = in.ai; g.ldb = in.lda;
    g.cr = M->G.re; g.ci = M->G.im; g.ldc = n;
    g.k_scale = ks; g.k_div = 1;
    g.herm_out = 1;
    g.tag = "gram";
    zgemm(g, 0, s);
  }
  // eigenvectors (conjugated, as rows) and eigenvalues of G
  const double* rows_r;
  const double* rows_i;
  static const bool no_sub = std::getenv("PTEBD_NO_SUBSPACE") != nullptr;   // debugging aid
  // The kept count follows the bond dimension before the gate, which the
  // warm rows carry: the subspace is sized for that count with a margin
  // rather than for chi_max (a subspace far wider than the kept values
  // spends its iterations on rounding-level eigenvalues without a gap), and
  // widened to chi_max when more values turn out to be kept.
  const int keep_full = std::min(M->chi_max, r);
  // the randomised route ignores the warm start: every basis starts from random rows
  WarmStart warm = in.warm;
  if (M->opts.svd == TEBD_SVD_RANDOMIZED) warm.kind = 0;
  int kw = 0;
  if (warm.kind == 1 && warm.src_rows == r) kw = warm.src_cols;
  if (warm.kind == 2 && warm.src_cols == r) kw = warm.src_rows;
  int keep = kw > 0 ? std::min(keep_full, kw + std::max(16, kw / 8)) : keep_full;
  int k = -1;
  bool wide = false;
  while (k < 0) {
    const int p = (M->sub_p > 0 && !no_sub) ? subspace_width_keep(r, keep, wide) : 0;
    bool sub_ok = p > 0 && p <= M->sub_p &&
                  subspace_topk(M, M->G.re, M->G.im, r, p, keep, warm, wide ? kWideIters : kNarrowIters);
    if (!sub_ok && !wide && p > 0) {
      const int pw = subspace_width_keep(r, keep, true);
      if (pw > 0 && pw <= M->sub_p) {
        if (debug_enabled()) std::fprintf(stderr, "[ptebd] subspace r=%d: narrow basis p=%d failed, wide p=%d\n", r, p, pw);
        wide = true;
        continue;
      }
    }
    if (sub_ok) {
      // the ledger is charged once the width is known to be enough
      double* trial = M->info_d + 12;
      fill_zero(trial, 1, s);
      select_truncate(M->norms, p, 1, M->chi_max, w_max, eps_g, lam_out, M->perm, M->inv_sig, kdev, nrm, trial,
                      M->info_d + 5, s);
      PTEBD_HIP(hipMemcpyAsync(M->h_info, kdev, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
      PTEBD_HIP(hipMemcpyAsync(M->h_part, nrm + 13, sizeof(double), hipMemcpyDeviceToHost, s));
      PTEBD_HIP(hipStreamSynchronize(s));
      if (M->h_info[0] > keep && keep < keep_full) {
        keep = keep_full;
        continue;
      }
      accumulate_slots(trial, 1, M->ledger, s);
      k = M->h_info[0];
      count_rule(M);
      rows_r = M->sZ.re;
      rows_i = M->sZ.im;
    } else {
      run_herm_jacobi(M, M->G.re, M->G.im, r, r, M->W.re, M->W.im, r);
      herm_diag(M->G.re, r, r, M->norms, s);
      select_truncate(M->norms, r, 1, M->chi_max, w_max, eps_g, lam_out, M->perm, M->inv_sig, kdev, nrm, M->ledger,
                      nullptr, s);
      PTEBD_HIP(hipMemcpyAsync(M->h_info, kdev, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
      PTEBD_HIP(hipMemcpyAsync(M->h_part, nrm + 13, sizeof(double), hipMemcpyDeviceToHost, s));
      PTEBD_HIP(hipStreamSynchronize(s));
      k = M->h_info[0];
      count_rule(M);
      rows_r = M->W.re;
      rows_i = M->W.im;
    }
  }
  if (left) {
    // V^+ = S^-1 U_k^+ diag(rs) A
    gather_rows(rows_r, rows_i, r, M->perm, M->inv_sig, k, m, xbuf.re, xbuf.im, m, kdev, s);
    ZGemmArgs v;
    v.m = k; v.n = n; v.k = m;
    v.ar = xbuf.re; v.ai = xbuf.im; v.lda = m;
    v.br = in.ar; v.bi = in.ai; v.ldb = in.lda;
    v.cr = vhr; v.ci = vhi; v.ldc = n;
    v.k_scale = in.rs; v.k_div = in.rdiv;
    v.tag = "svd_project";
    zgemm(v, 0, s);
    // smallest kept over largest Schmidt value (read back with k)
    if (k >= 2 && M->h_part[0] < kRefineRatio) cholqr_rows(M, vhr, vhi, n, k, n, xbuf);
  } else {
    // eigenvectors of A^+ A are the right singular vectors
    gather_rows(rows_r, rows_i, r, M->perm, nullptr, k, n, vhr, vhi, n, kdev, s);
  }
  return k;
}

// U(1) block-sparse truncated SVD (Sec. II B: the tensors are kept in
// particle-number sectors).  With the rows and columns of A grouped by their
// particle number, diag(rs) A is block diagonal, so its singular triplets are
// those of the blocks: each block is gathered into xbuf and decomposed on its
// own (Jacobi: one-sided Jacobi on the rows of the block or of its conjugate
// transpose; Gram: the smaller Gram matrix of the block and its eigenpairs),
// and the truncation rule runs once over the union of the sector spectra, so
// that the kept values, the discarded weight and the ledger are those of the
// dense SVD.  The kept rows of V^+ are scattered back to the dense column
// positions; every other entry of the output rows is zero.
int svd_trunc_u1(tebd_mps* M, const SvdIn& in, const std::vector<int>& rq, const std::vector<int>& cq,
                 double* lam_out, double* vhr, double* vhi, int slot, tebd_mps::Z xbuf, std::vector<int>& kept_q) {
  hipStream_t s = M->stream;
  const int m = in.m, n = in.n;
  const bool gram = M->opts.svd != TEBD_SVD_JACOBI;
  double* nrm = M->info_d + 2 * slot;
  int* kdev = M->info_i + slot;
  const double eps = M->opts.trunc_rel;   // >= TEBD_GRAM_EPS_MIN on the Gram route (checked at creation)
  const double w_max = M->opts.trunc_weight;
  struct Sector {
    int q = 0;
    std::vector<int> rows, cols;
    int m = 0, n = 0, r = 0;
    bool left = true;        // decompose the block itself (Jacobi on its rows, Gram B B^+), else its conjugate transpose
    int64_t off = 0;         // block in xbuf
    int64_t goff = 0;        // r x r Gram / eigenvector rows / rotations in G and W
    int u0 = 0;              // first value of the sector in the union
    int64_t ro = 0, co = 0;  // row and column lists in u_idx
    std::vector<int> kept;   // ranks (by decreasing value) of the kept values
    int64_t xoff = 0, yoff = 0;
  };
  std::map<int, Sector> by_q;
  for (int r = 0; r < m; ++r) by_q[rq[r]].rows.push_back(r);
  for (int c = 0; c < n; ++c) {
    auto it = by_q.find(cq[c]);
    if (it != by_q.end()) it->second.cols.push_back(c);
  }
  std::vector<Sector*> secs;
  int64_t off = 0, goff = 0, io = 0;
  int nvals = 0;
  M->h_idx.clear();
  for (auto& kv : by_q) {
    Sector& S = kv.second;
    if (S.cols.empty()) continue;   // rows of this number meet no column: they are zero
    S.q = kv.first;
    S.m = (int)S.rows.size();
    S.n = (int)S.cols.size();
    S.r = std::min(S.m, S.n);
    S.left = in.prefer_right ? (S.m < S.n) : (S.m <= S.n);
    S.off = off;
    off += (int64_t)S.m * S.n;
    S.goff = goff;
    goff += (int64_t)S.r * S.r;
    S.u0 = nvals;
    nvals += S.r;
    S.ro = io;
    M->h_idx.insert(M->h_idx.end(), S.rows.begin(), S.rows.end());
    io += S.m;
    S.co = io;
    M->h_idx.insert(M->h_idx.end(), S.cols.begin(), S.cols.end());
    io += S.n;
    secs.push_back(&S);
  }
  if (secs.empty()) throw Error(-1, "U(1) SVD: no particle-number sector has both rows and columns");
  if (io + std::min(m, n) > M->u_idx_cap) throw Error(-1, "U(1) SVD: sector lists exceed their buffer");
  PTEBD_HIP(hipMemcpyAsync(M->u_idx, M->h_idx.data(), sizeof(int) * io, hipMemcpyHostToDevice, s));
  const int64_t idx_end = io;
  // gather every sector block (Gram: as it stands; Jacobi: rows, or the
  // conjugate transpose for a tall block); the Jacobi route decomposes all
  // sectors in one batched run
  std::vector<JacobiArgs> jac;
  for (Sector* S : secs) {
    const int* rows = M->u_idx + S->ro;
    const int* cols = M->u_idx + S->co;
    double* br = xbuf.re + S->off;
    double* bi = xbuf.im + S->off;
    double* wr = M->W.re + S->goff;
    double* wi = M->W.im + S->goff;
    if (!gram) {
      if (S->left) {
        // rows of the block become sigma_i v_i^+
        gather_block(in.ar, in.ai, in.lda, in.rs, in.rdiv, rows, S->m, cols, S->n, 0, br, bi, S->n, s);
        if (S->m > 1)
          jac.push_back(jacobi_args(br, bi, S->n, nullptr, nullptr, 0, S->m, S->n, jacobi_tol(S->n), 0.0));
      } else {
        // rows of the conjugate transpose (n x m) become sigma_i u_i^+; the
        // accumulated rotations are the rows v_i^+
        gather_block(in.ar, in.ai, in.lda, in.rs, in.rdiv, rows, S->m, cols, S->n, 1, br, bi, S->m, s);
        if (S->n > 1)
          jac.push_back(jacobi_args(br, bi, S->m, wr, wi, S->n, S->n, S->m, jacobi_tol(S->m), 0.0));
        else
          set_identity(wr, wi, 1, 1, s);
      }
    } else {
      gather_block(in.ar, in.ai, in.lda, in.rs, in.rdiv, rows, S->m, cols, S->n, 0, br, bi, S->n, s);
    }
  }
  if (!jac.empty()) run_jacobi_batched(M, jac);
  // The Gram matrix of every sector, packed r x r blocks.
  auto sector_grams = [&]() {
    for (Sector* S : secs) {
      const double* br = xbuf.re + S->off;
      const double* bi = xbuf.im + S->off;
      ZGemmArgs g;
      if (S->left) {   // B B^+ (m x m)
        g.m = S->m; g.n = S->m; g.k = S->n;
        g.ar = br; g.ai = bi; g.lda = S->n;
        g.br = br; g.bi = bi; g.ldb = S->n; g.transB = 1;
      } else {         // B^+ B (n x n)
        g.m = S->n; g.n = S->n; g.k = S->m;
        g.ar = br; g.ai = bi; g.lda = S->n; g.transA = 1;
        g.br = br; g.bi = bi; g.ldb = S->n;
      }
      g.cr = M->G.re + S->goff; g.ci = M->G.im + S->goff; g.ldc = S->r;
      g.herm_out = 1;
      g.tag = "u1_gram";
      zgemm(g, 0, s);
    }
  };
  if (gram) {
    sector_grams();
    std::vector<BatchItem> items;
    for (Sector* S : secs) {
      double* wr = M->W.re + S->goff;
      double* wi = M->W.im + S->goff;
      if (S->r > 1)
        items.push_back(BatchItem{M->G.re + S->goff, M->G.im + S->goff, wr, wi, S->r});
      else
        set_identity(wr, wi, 1, 1, s);
    }
    // all sector eigenproblems in one batched Jacobi
    if (!items.empty()) run_herm_jacobi_batched(M, items);
  }
  // the union of the sector spectra (after every Jacobi run, which uses
  // M->norms as its own scratch)
  for (Sector* S : secs) {
    double* out = M->norms + S->u0;
    if (!gram) {
      if (S->left)
        row_norms(xbuf.re + S->off, xbuf.im + S->off, S->n, S->m, S->n, out, s);
      else
        row_norms(xbuf.re + S->off, xbuf.im + S->off, S->m, S->n, S->m, out, s);
    } else {
      herm_diag(M->G.re + S->goff, S->r, S->r, out, s);
    }
  }
  select_truncate(M->norms, nvals, gram ? 1 : 0, M->chi_max, w_max, eps, lam_out, M->perm, M->inv_sig, kdev, nrm,
                  M->ledger, nullptr, s);
  PTEBD_HIP(hipMemcpyAsync(M->h_info, kdev, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
  PTEBD_HIP(hipMemcpyAsync(M->h_part, nrm + 13, sizeof(double), hipMemcpyDeviceToHost, s));
  PTEBD_HIP(hipStreamSynchronize(s));
  const double kept_ratio = M->h_part[0];
  const int k = M->h_info[0];
  count_rule(M);
  M->h_perm.resize(k);
  PTEBD_HIP(hipMemcpyAsync(M->h_perm.data(), M->perm, sizeof(int) * k, hipMemcpyDeviceToHost, s));
  PTEBD_HIP(hipStreamSynchronize(s));
  {
    std::vector<int> u0s;
    for (Sector* S : secs) u0s.push_back(S->u0);
    for (int i = 0; i < k; ++i) {
      const int v = M->h_perm[i];
      const int si = (int)(std::upper_bound(u0s.begin(), u0s.end(), v) - u0s.begin()) - 1;
      if (si < 0 || v >= secs[si]->u0 + secs[si]->r) throw Error(-3, "U(1) SVD: kept value outside every sector");
      secs[si]->kept.push_back(i);
    }
  }
  // output order: by particle number, then by rank
  kept_q.clear();
  M->h_order.clear();
  for (Sector* S : secs)
    for (int i : S->kept) {
      M->h_order.push_back(i);
      kept_q.push_back(S->q);
    }
  if (idx_end + k > M->u_idx_cap) throw Error(-1, "U(1) SVD: sector lists exceed their buffer");
  int* d_order = M->u_idx + idx_end;
  PTEBD_HIP(hipMemcpyAsync(d_order, M->h_order.data(), sizeof(int) * k, hipMemcpyHostToDevice, s));
  take(lam_out, d_order, k, M->sq, s);
  PTEBD_HIP(hipMemcpyAsync(lam_out, M->sq, sizeof(double) * k, hipMemcpyDeviceToDevice, s));
  // row-copy table: for the left Gram blocks the scaled eigenvector rows
  // S^-1 U^+ of every sector first (into G, free by now), then the output rows
  M->h_tab.clear();
  int nx = 0;
  if (gram) {
    int64_t xo = 0, yo = 0;
    for (Sector* S : secs) {
      if (!S->left || S->kept.empty()) continue;
      S->xoff = xo;
      S->yoff = yo;
      for (size_t t = 0; t < S->kept.size(); ++t) {
        const int i = S->kept[t];
        const int64_t loc = M->h_perm[i] - S->u0;
        M->h_tab.push_back(RowCopy{M->W.re + S->goff + loc * S->r, M->W.im + S->goff + loc * S->r,
                                   M->G.re + xo + (int64_t)t * S->m, M->G.im + xo + (int64_t)t * S->m, nullptr,
                                   (int64_t)S->m, (int64_t)i});
      }
      xo += (int64_t)S->kept.size() * S->m;
      yo += (int64_t)S->kept.size() * S->n;
    }
    nx = (int)M->h_tab.size();
  }
  int64_t o = 0;
  for (Sector* S : secs) {
    for (size_t t = 0; t < S->kept.size(); ++t, ++o) {
      const int i = S->kept[t];
      const int64_t loc = M->h_perm[i] - S->u0;
      const double* sr;
      const double* si;
      int64_t sidx = -1;
      if (!gram && S->left) {
        sr = xbuf.re + S->off + loc * S->n;
        si = xbuf.im + S->off + loc * S->n;
        sidx = i;
      } else if (gram && S->left) {
        sr = M->uv.re + S->yoff + (int64_t)t * S->n;
        si = M->uv.im + S->yoff + (int64_t)t * S->n;
      } else {   // rows of W: eigenvector rows (right Gram) or accumulated rotations (tall Jacobi block)
        sr = M->W.re + S->goff + loc * S->r;
        si = M->W.im + S->goff + loc * S->r;
      }
      M->h_tab.push_back(RowCopy{sr, si, vhr + o * n, vhi + o * n, M->u_idx + S->co, (int64_t)S->n, sidx});
    }
  }
  if ((int64_t)M->h_tab.size() > M->u_tab_cap) throw Error(-1, "U(1) SVD: row table exceeds its buffer");
  PTEBD_HIP(hipMemcpyAsync(M->u_tab, M->h_tab.data(), sizeof(RowCopy) * M->h_tab.size(), hipMemcpyHostToDevice, s));
  if (nx > 0) {
    rows_copy(M->u_tab, nx, M->inv_sig, s);
    for (Sector* S : secs) {
      if (!S->left || S->kept.empty()) continue;
      ZGemmArgs v;   // V^+ rows of the sector = (S^-1 U^+) B
      v.m = (int)S->kept.size(); v.n = S->n; v.k = S->m;
      v.ar = M->G.re + S->xoff; v.ai = M->G.im + S->xoff; v.lda = S->m;
      v.br = xbuf.re + S->off; v.bi = xbuf.im + S->off; v.ldb = S->n;
      v.cr = M->uv.re + S->yoff; v.ci = M->uv.im + S->yoff; v.ldc = S->n;
      v.tag = "u1_project";
      zgemm(v, 0, s);
    }
  }
  fill_zero(vhr, (int64_t)k * n, s);
  fill_zero(vhi, (int64_t)k * n, s);
  rows_copy(M->u_tab + nx, k, M->inv_sig, s);
  // Gram route: the rows of different sectors are orthogonal exactly
  // (disjoint columns), and within a sector they are in decreasing order of
  // value, which is the order Cholesky-QR needs
  if (gram && k >= 2 && kept_ratio < kRefineRatio) cholqr_rows(M, vhr, vhi, n, k, n, xbuf);
  // the host tables stay untouched until the next call, which synchronises first
  return k;
}

std::vector<std::vector<int>> infer_charges(const tebd_mps* M, const int* chi, const double* B) {
  const int L = M->L, d = M->d;
  std::vector<std::vector<int>> q(L + 1);
  q[0].assign(1, 0);
  int64_t off = 0;
  for (int i = 0; i < L; ++i) {
    const int cl = chi[i], cr = chi[i + 1];
    const int64_t nel = (int64_t)cl * d * cr;
    const double* re = B + off;
    const double* im = B + off + nel;
    std::vector<int> qr(cr, 0);
    std::vector<char> seen(cr, 0);
    for (int a = 0; a < cl; ++a)
      for (int t = 0; t < d; ++t)
        for (int b = 0; b < cr; ++b) {
          const int64_t e = ((int64_t)a * d + t) * cr + b;
          if (re[e] == 0.0 && im[e] == 0.0) continue;
          const int v = q[i][a] + M->qs[t];
          if (!seen[b]) {
            seen[b] = 1;
            qr[b] = v;
          } else if (qr[b] != v) {
            throw Error(-1, "state has no definite particle number on bond " + std::to_string(i + 1) + " index " +
                                std::to_string(b));
          }
        }
    for (int b = 0; b < cr; ++b)
      if (!seen[b])
        throw Error(-1, "bond " + std::to_string(i + 1) + " index " + std::to_string(b) +
                            " is reached by no non-zero entry of its left tensor");
    q[i + 1] = std::move(qr);
    off += 2 * nel;
  }
  return q;
}

TileTuner& tile_tuner() {
  static TileTuner t;
  return t;
}

namespace {

bool autotune_enabled() {
  static const bool v = std::getenv("PTEBD_NO_AUTOTUNE") == nullptr;
  return v;
}

// A theta or gate product with the tile shape the tuner picked for its
// (device, m, n, k, batch).  A shape seen for the first time is run three
// times with each FP64 tile on the worker's stream (the products overwrite
// their output and read only their inputs, so the repetitions leave the
// result as one launch would) and the faster tile is kept for the life of
// the process, for every handle.  Both tiles accumulate every output element
// in the same K order, so the choice does not change the result.  FP32
// products have one tile shape.
void tuned_gemm(ZGemmArgs g, int prec, hipStream_t s) {
  ptebd::TileTuner& T = tile_tuner();
  if (prec != 0 || !autotune_enabled() || g.beta) {
    zgemm(g, prec, s);
    return;
  }
  int dev = 0;
  PTEBD_HIP(hipGetDevice(&dev));
  const std::array<int64_t, 5> key{dev, g.m, g.n, g.k, g.batch};
  {
    std::lock_guard<std::mutex> lk(T.mu);
    auto it = T.best.find(key);
    if (it != T.best.end()) {
      g.tile = it->second;
      (g.tile == 128 ? T.launches_128 : T.launches_64) += 1;
    }
  }
  if (g.tile) {
    zgemm(g, prec, s);
    return;
  }
  hipEvent_t e[3];
  for (auto& x : e) PTEBD_HIP(hipEventCreate(&x));
  float ms[2] = {0.f, 0.f};
  const int tiles[2] = {64, 128};
  for (int v = 0; v < 2; ++v) {
    g.tile = tiles[v];
    zgemm(g, prec, s);   // warm
    PTEBD_HIP(hipEventRecord(e[0], s));
    for (int r = 0; r < 3; ++r) zgemm(g, prec, s);
    PTEBD_HIP(hipEventRecord(e[1], s));
    PTEBD_HIP(hipEventSynchronize(e[1]));
    PTEBD_HIP(hipEventElapsedTime(&ms[v], e[0], e[1]));
  }
  for (auto& x : e) PTEBD_HIP(hipEventDestroy(x));
  const int pick = ms[1] < ms[0] ? 128 : 64;
  std::lock_guard<std::mutex> lk(T.mu);
  if (T.best.emplace(key, pick).second) ++T.shapes_tuned;
  if (debug_enabled())
    std::fprintf(stderr, "[ptebd] tile tuner m=%ld n=%ld k=%ld batch=%ld: 64 %.3f ms, 128 %.3f ms -> %d\n",
                 (long)g.m, (long)g.n, (long)g.k, (long)g.batch, ms[0] / 3, ms[1] / 3, pick);
}

// theta = B_j B_{j+1} B_{j+2} into W->psi and psi' = G psi, batched over
// the left bond index, into W->psip (Sec. II B).
void theta_gate(tebd_mps* S, tebd_mps* W, int j, std::pair<double*, double*> G, hipStream_t s) {
  const int d = W->d, d3 = d * d * d;
  const int cl = S->chi[j], c1 = S->chi[j + 1], c2 = S->chi[j + 2], cr = S->chi[j + 3];
  const int prec = W->opts.prec;
  {  // T1 = B_j B_{j+1}
    ZGemmArgs g;
    g.m = cl * d; g.n = d * c2; g.k = c1;
    g.ar = S->Br[j]; g.ai = S->Bi[j]; g.lda = c1;
    g.br = S->Br[j + 1]; g.bi = S->Bi[j + 1]; g.ldb = (int64_t)d * c2;
    g.cr = W->T1.re; g.ci = W->T1.im; g.ldc = (int64_t)d * c2;
    g.tag = "theta";
    tuned_gemm(g, prec, s);
  }
  {  // psi = T1 B_{j+2}
    ZGemmArgs g;
    g.m = cl * d * d; g.n = d * cr; g.k = c2;
    g.ar = W->T1.re; g.ai = W->T1.im; g.lda = c2;
    g.br = S->Br[j + 2]; g.bi = S->Bi[j + 2]; g.ldb = (int64_t)d * cr;
    g.cr = W->psi.re; g.ci = W->psi.im; g.ldc = (int64_t)d * cr;
    g.tag = "theta";
    tuned_gemm(g, prec, s);
  }
  {  // psi'[a] = G psi[a]
    ZGemmArgs g;
    g.m = d3; g.n = cr; g.k = d3; g.batch = cl;
    g.ar = G.first; g.ai = G.second; g.lda = d3; g.sA = 0;
    g.br = W->psi.re; g.bi = W->psi.im; g.ldb = cr; g.sB = (int64_t)d3 * cr;
    g.cr = W->psip.re; g.ci = W->psip.im; g.ldc = cr; g.sC = (int64_t)d3 * cr;
    g.tag = "gate";
    tuned_gemm(g, prec, s);
  }
}

// B_j = psi' V1 / |S1| (m1 x k1); the Jacobi route divides by the norm of
// the kept values on the device (info_d[0]).
void update_left_jacobi(tebd_mps* S, tebd_mps* W, int j, int m1, int n1, int k1, hipStream_t s) {
  ZGemmArgs g;
  g.m = m1; g.n = k1; g.k = n1;
  g.ar = W->psip.re; g.ai = W->psip.im; g.lda = n1;
  g.br = W->V1h.re; g.bi = W->V1h.im; g.ldb = n1; g.transB = 1;
  g.cr = S->Br[j]; g.ci = S->Bi[j]; g.ldc = k1;
  g.alpha_dev = W->info_d + 0;
  g.alpha_recip = 1;
  g.tag = "update_left";
  zgemm(g, 0, s);
}

// B_{j+1} = V1^+ V2 / |S2| (m2 x k2), V2^+ already in B_{j+2}.
void update_middle_jacobi(tebd_mps* S, tebd_mps* W, int j, int m2, int n2, int k2, hipStream_t s) {
  ZGemmArgs g;
  g.m = m2; g.n = k2; g.k = n2;
  g.ar = W->V1h.re; g.ai = W->V1h.im; g.lda = n2;
  g.br = S->Br[j + 2]; g.bi = S->Bi[j + 2]; g.ldb = n2; g.transB = 1;
  g.cr = S->Br[j + 1]; g.ci = S->Bi[j + 1]; g.ldc = k2;
  g.alpha_dev = W->info_d + 2;
  g.alpha_recip = 1;
  g.tag = "update_middle";
  zgemm(g, 0, s);
}

// One gate on sites (j, j+1, j+2) of the state held by S, with the buffers,
// stream and settings of worker W.
void gate_update(tebd_mps* S, tebd_mps* W, int j, std::pair<double*, double*> G) {
  hipStream_t s = W->stream;
  const int d = W->d;
  const int cl = S->chi[j], c1 = S->chi[j + 1], c2 = S->chi[j + 2], cr = S->chi[j + 3];
  theta_gate(S, W, j, G, s);
  const int m1 = cl * d, n1 = d * d * cr;
  SvdIn in1{W->psip.re, W->psip.im, n1, m1, n1, S->lam[j], d};
  // before the gate the left singular space of theta across bond j+1 is
  // spanned by the columns of Lambda_j B_j
  in1.warm.kind = 1;
  in1.warm.sr = S->Br[j]; in1.warm.si = S->Bi[j]; in1.warm.ld = c1;
  in1.warm.src_rows = m1; in1.warm.src_cols = c1;
  in1.warm.rs = S->lam[j]; in1.warm.rdiv = d;
  std::vector<int> q1, q2;
  int k1;
  if (S->u1) {
    // rows (a, s1) hold q_j[a] + s1 bosons left of bond j+1; columns
    // (s2, s3, b) hold q_{j+3}[b] - s2 - s3
    const std::vector<int>& ql = S->q[j];
    const std::vector<int>& qr = S->q[j + 3];
    std::vector<int> rq((size_t)m1), cq((size_t)n1);
    for (int a = 0; a < cl; ++a)
      for (int t = 0; t < d; ++t) rq[(size_t)a * d + t] = ql[a] + S->qs[t];
    for (int t2 = 0; t2 < d; ++t2)
      for (int t3 = 0; t3 < d; ++t3)
        for (int b = 0; b < cr; ++b) cq[((size_t)t2 * d + t3) * cr + b] = qr[b] - S->qs[t2] - S->qs[t3];
    k1 = svd_trunc_u1(W, in1, rq, cq, S->lam[j + 1], W->V1h.re, W->V1h.im, 0, W->psi, q1);
  } else {
    k1 = svd_trunc(W, in1, S->lam[j + 1], W->V1h.re, W->V1h.im, 0, W->psi);
  }
  const bool gram = W->opts.svd != TEBD_SVD_JACOBI;
  if (!gram) {
    update_left_jacobi(S, W, j, m1, n1, k1, s);
  } else {  // B_j = psi' V1 / |S1|
    ZGemmArgs g;
    g.m = m1; g.n = k1; g.k = n1;
    g.ar = W->psip.re; g.ai = W->psip.im; g.lda = n1;
    g.br = W->V1h.re; g.bi = W->V1h.im; g.ldb = n1; g.transB = 1;
    g.cr = S->Br[j]; g.ci = S->Bi[j]; g.ldc = k1;
    g.tag = "update_left";
    zgemm(g, 0, s);
    // Gram route: Lambda_j psi' V1 = U1 S1 gives each Schmidt value as a column
    // norm to the rounding of the product, where the Gram eigenvalue s^2 only
    // resolves s to u / s (the division by |S1| follows)
    refine_sigma(S->Br[j], S->Bi[j], k1, m1, k1, S->lam[j], d, W->part, W->part_cap, S->lam[j + 1], W->info_d + 0,
                 s);
  }
  const int m2 = k1 * d, n2 = d * cr;
  SvdIn in2{W->V1h.re, W->V1h.im, n2, m2, n2, S->lam[j + 1], d};
  // before the gate the right singular space across bond j+2 is the row
  // space of B_{j+2}
  in2.prefer_right = true;
  in2.warm.kind = 2;
  in2.warm.sr = S->Br[j + 2]; in2.warm.si = S->Bi[j + 2]; in2.warm.ld = n2;
  in2.warm.src_rows = c2; in2.warm.src_cols = n2;
  int k2;
  if (S->u1) {
    // rows (a', s2): q1[a'] + s2; columns (s3, b): q_{j+3}[b] - s3
    const std::vector<int>& qr = S->q[j + 3];
    std::vector<int> rq((size_t)m2), cq((size_t)n2);
    for (int a = 0; a < k1; ++a)
      for (int t = 0; t < d; ++t) rq[(size_t)a * d + t] = q1[a] + S->qs[t];
    for (int t3 = 0; t3 < d; ++t3)
      for (int b = 0; b < cr; ++b) cq[(size_t)t3 * cr + b] = qr[b] - S->qs[t3];
    k2 = svd_trunc_u1(W, in2, rq, cq, S->lam[j + 2], S->Br[j + 2], S->Bi[j + 2], 1, W->X2, q2);
  } else {
    k2 = svd_trunc(W, in2, S->lam[j + 2], S->Br[j + 2], S->Bi[j + 2], 1, W->X2);
  }
  if (!gram) {
    update_middle_jacobi(S, W, j, m2, n2, k2, s);
  } else {  // B_{j+1} = V1^+ V2 / |S2|
    ZGemmArgs g;
    g.m = m2; g.n = k2; g.k = n2;
    g.ar = W->V1h.re; g.ai = W->V1h.im; g.lda = n2;
    g.br = S->Br[j + 2]; g.bi = S->Bi[j + 2]; g.ldb = n2; g.transB = 1;
    g.cr = S->Br[j + 1]; g.ci = S->Bi[j + 1]; g.ldc = k2;
    g.tag = "update_middle";
    zgemm(g, 0, s);
    // S1 V1^+ V2 = U2 S2 (as above)
    refine_sigma(S->Br[j + 1], S->Bi[j + 1], k2, m2, k2, S->lam[j + 1], d, W->part, W->part_cap, S->lam[j + 2],
                 W->info_d + 2, s);
  }
  S->chi[j + 1] = k1;
  S->chi[j + 2] = k2;
  if (S->u1) {
    S->q[j + 1] = std::move(q1);
    S->q[j + 2] = std::move(q2);
  }
}

// Two-site gate on super sites (K, K+1) (Sec. II B, d_eff = D = d^2):
//   psi  = B_K B_{K+1}                     (chi_l D) x (D chi_r)        GEMM
//   psi' = G psi (batched over chi_l)      D^2 x chi_r per left index   GEMM
//   SVD of Lambda_K psi' as (chi_l D) x (D chi_r), truncate -> k
//   B_K = psi' V / |S|,  B_{K+1} = V^+,  Lambda_{K+1} = S / |S|.
void gate_update2(tebd_mps* S, tebd_mps* W, int K, std::pair<double*, double*> G) {
  hipStream_t s = W->stream;
  const int D = W->d, D2 = D * D;
  const int cl = S->chi[K], cm = S->chi[K + 1], cr = S->chi[K + 2];
  const int prec = W->opts.prec;
  {  // psi = B_K B_{K+1}
    ZGemmArgs g;
    g.m = cl * D; g.n = D * cr; g.k = cm;
    g.ar = S->Br[K]; g.ai = S->Bi[K]; g.lda = cm;
    g.br = S->Br[K + 1]; g.bi = S->Bi[K + 1]; g.ldb = (int64_t)D * cr;
    g.cr = W->psi.re; g.ci = W->psi.im; g.ldc = (int64_t)D * cr;
    g.tag = "theta";
    tuned_gemm(g, prec, s);
  }
  {  // psi'[a] = G psi[a]
    ZGemmArgs g;
    g.m = D2; g.n = cr; g.k = D2; g.batch = cl;
    g.ar = G.first; g.ai = G.second; g.lda = D2; g.sA = 0;
    g.br = W->psi.re; g.bi = W->psi.im; g.ldb = cr; g.sB = (int64_t)D2 * cr;
    g.cr = W->psip.re; g.ci = W->psip.im; g.ldc = cr; g.sC = (int64_t)D2 * cr;
    g.tag = "gate";
    tuned_gemm(g, prec, s);
  }
  const int m1 = cl * D, n1 = D * cr;
  SvdIn in{W->psip.re, W->psip.im, n1, m1, n1, S->lam[K], D};
  // before the gate the left singular space across bond K+1 is spanned by
  // the columns of Lambda_K B_K
  in.warm.kind = 1;
  in.warm.sr = S->Br[K]; in.warm.si = S->Bi[K]; in.warm.ld = cm;
  in.warm.src_rows = m1; in.warm.src_cols = cm;
  in.warm.rs = S->lam[K]; in.warm.rdiv = D;
  // V^+ goes straight to B_{K+1}: psi' no longer needs the old B_{K+1}
  std::vector<int> qk;
  int k;
  if (S->u1) {
    // rows (a, s1): q_K[a] + bosons of s1; columns (s2, b): q_{K+2}[b] - bosons of s2
    const std::vector<int>& ql = S->q[K];
    const std::vector<int>& qr = S->q[K + 2];
    std::vector<int> rq((size_t)m1), cq((size_t)n1);
    for (int a = 0; a < cl; ++a)
      for (int t = 0; t < D; ++t) rq[(size_t)a * D + t] = ql[a] + S->qs[t];
    for (int t = 0; t < D; ++t)
      for (int b = 0; b < cr; ++b) cq[(size_t)t * cr + b] = qr[b] - S->qs[t];
    k = svd_trunc_u1(W, in, rq, cq, S->lam[K + 1], S->Br[K + 1], S->Bi[K + 1], 0, W->psi, qk);
  } else {
    k = svd_trunc(W, in, S->lam[K + 1], S->Br[K + 1], S->Bi[K + 1], 0, W->psi);
  }
  {  // B_K = psi' V / |S|
    ZGemmArgs g;
    g.m = m1; g.n = k; g.k = n1;
    g.ar = W->psip.re; g.ai = W->psip.im; g.lda = n1;
    g.br = S->Br[K + 1]; g.bi = S->Bi[K + 1]; g.ldb = n1; g.transB = 1;
    g.cr = S->Br[K]; g.ci = S->Bi[K]; g.ldc = k;
    const bool gram = W->opts.svd != TEBD_SVD_JACOBI;
    if (!gram) {
      g.alpha_dev = W->info_d + 0;
      g.alpha_recip = 1;
    }
    g.tag = "update_left";
    zgemm(g, 0, s);
    // Lambda_K psi' V = U S: Schmidt values as column norms (Gram route)
    if (gram) refine_sigma(S->Br[K], S->Bi[K], k, m1, k, S->lam[K], D, W->part, W->part_cap, S->lam[K + 1],
                           W->info_d + 0, s);
  }
  S->chi[K + 1] = k;
  if (S->u1) S->q[K + 1] = std::move(qk);
}

void update_gate(tebd_mps* S, tebd_mps* W, int j, std::pair<double*, double*> G) {
  if (S->super)
    gate_update2(S, W, j, G);
  else
    gate_update(S, W, j, G);
}

// One gate's Jacobi-route SVD of diag(rs) A, split into the steps a fused
// layer interleaves with the other gates' SVDs.  The calls, arguments and
// order are those of svd_trunc's Jacobi branch.
struct JacSvd {
  tebd_mps* W = nullptr;   // workspace of the gate
  SvdIn in{};
  double* lam_out = nullptr;
  double* vhr = nullptr;
  double* vhi = nullptr;
  int slot = 0;
  tebd_mps::Z xbuf;
  int k = 0;
};

// Jacobi on the rows of A_s (m <= n), else on the rows of A_s^+ with the
// right singular vectors accumulated in W->W.
bool jac_rows(const SvdIn& in) { return in.m <= in.n; }

JacobiArgs jac_entry(const JacSvd& x) {
  const SvdIn& in = x.in;
  tebd_mps* W = x.W;
  JacobiArgs a =
      jac_rows(in)
          ? jacobi_args(x.xbuf.re, x.xbuf.im, in.n, nullptr, nullptr, 0, in.m, in.n, jacobi_tol(in.n), 0.0)
          : jacobi_args(x.xbuf.re, x.xbuf.im, in.m, W->W.re, W->W.im, in.n, in.n, in.m, jacobi_tol(in.m), 0.0);
  if (jacobi_part(a) > W->part_cap) throw Error(-1, "Jacobi scratch too small");
  a.part = W->part;
  return a;
}

// The arguments of every small step of x's SVD (staging, row norms, the
// Jacobi prologue, selection, gathering), as svd_trunc's Jacobi branch
// passes them to the single-matrix launchers; kout receives k and the rule.
FusedSvdArgs fused_args(const JacSvd& x, int* kout) {
  const SvdIn& in = x.in;
  tebd_mps* W = x.W;
  const bool rows = jac_rows(in);
  FusedSvdArgs f{};
  f.xr = in.ar; f.xi = in.ai; f.ldx = in.lda;
  f.rs = in.rs; f.rdiv = in.rdiv;
  f.rows = in.m; f.cols = in.n; f.transpose = rows ? 0 : 1;
  f.yr = x.xbuf.re; f.yi = x.xbuf.im; f.ldy = rows ? in.n : in.m;
  f.r = rows ? in.m : in.n;
  f.c = rows ? in.n : in.m;
  f.norms = W->norms;
  f.wr = rows ? nullptr : W->W.re;
  f.wi = rows ? nullptr : W->W.im;
  f.ldw = in.n;
  int np2 = 1;
  while (np2 < f.r) np2 <<= 1;
  f.npow2 = np2;
  f.is_gram = 0;
  f.chi_max = W->chi_max;
  f.w_max = W->opts.trunc_weight;
  f.eps = W->opts.trunc_rel;
  f.extra_tail = nullptr;
  f.lam_out = x.lam_out; f.perm = W->perm; f.inv_sig = W->inv_sig;
  f.info_i = W->info_i + x.slot; f.info_d = W->info_d + 2 * x.slot; f.ledger = W->ledger;
  f.kout = kout;
  f.gr = rows ? x.xbuf.re : W->W.re;
  f.gi = rows ? x.xbuf.im : W->W.im;
  f.ldg = in.n;
  f.gscale = rows ? 1 : 0;
  f.gc = in.n;
  f.dr = x.vhr; f.di = x.vhi; f.ldd = in.n;
  return f;
}

// The SVDs of v (one per workspace) on the stream of R, in groups of up to
// kFusedMax: every small step is one launch for the whole group, the Jacobi
// sweeps run batched, and one read-back per group returns all truncation
// ranks.
void jac_batch(tebd_mps* R, std::vector<JacSvd>& v, hipStream_t s) {
  if (R->stream != s) throw Error(-3, "fused layer: the Jacobi runner must use the layer's stream");
  if (!R->f_tab || !R->u_batch) throw Error(-1, "fused layer: the runner has no batch tables");
  const size_t per = sizeof(JacobiArgs) + 2 * sizeof(int64_t) + 2 * sizeof(int) + sizeof(double);
  const size_t fit = std::min<size_t>(kFusedMax, R->u_batch_cap > 128 ? ((size_t)R->u_batch_cap - 128) / per : 0);
  if (fit == 0) throw Error(-1, "fused layer: no batched Jacobi tables");
  for (size_t g0 = 0; g0 < v.size(); g0 += fit) {
    const int cnt = (int)std::min(fit, v.size() - g0);
    int max_rows = 0, max_cols = 0, max_r = 0, max_np2 = 1;
    std::vector<JacobiArgs> tab;
    tab.reserve(cnt);
    for (int i = 0; i < cnt; ++i) {
      const JacSvd& x = v[g0 + i];
      FusedSvdArgs& f = R->h_ftab[i];
      f = fused_args(x, R->f_k + 2 * i);
      max_rows = std::max(max_rows, f.rows);
      max_cols = std::max(max_cols, f.cols);
      max_r = std::max(max_r, f.r);
      max_np2 = std::max(max_np2, f.npow2);
      tab.push_back(jac_entry(x));
    }
    PTEBD_HIP(hipMemcpyAsync(R->f_tab, R->h_ftab, sizeof(FusedSvdArgs) * cnt, hipMemcpyHostToDevice, s));
    fused_stage(R->f_tab, cnt, max_rows, max_cols, s);
    run_jacobi_group(R, tab, [&](double* tiny2) {
      fused_row_norms(R->f_tab, cnt, max_r, s);
      fused_jacobi_prologue(R->f_tab, cnt, max_r, tiny2, s);
    });
    fused_row_norms(R->f_tab, cnt, max_r, s);
    fused_select(R->f_tab, cnt, max_np2, s);
    PTEBD_HIP(hipMemcpyAsync(R->h_fk, R->f_k, sizeof(int) * 2 * cnt, hipMemcpyDeviceToHost, s));
    PTEBD_HIP(hipStreamSynchronize(s));
    int max_k = 0;
    for (int i = 0; i < cnt; ++i) {
      JacSvd& x = v[g0 + i];
      x.k = R->h_fk[2 * i];
      x.W->h_info[0] = x.k;
      x.W->h_info[4] = R->h_fk[2 * i + 1];
      count_rule(x.W);
      max_k = std::max(max_k, x.k);
    }
    fused_gather(R->f_tab, cnt, max_k, max_cols, s);
  }
}

// One gate of a fused layer: the state it acts on, the workspace it uses.
struct FusedJob {
  tebd_mps* M;
  tebd_mps* W;
  int j;
  std::pair<double*, double*> G;
};

// Gates on disjoint sites, each with a workspace of its own, in lockstep on
// stream s (Sec. I: the gates of a layer are independent): the theta and
// gate products of all of them are issued back to back, their SVDs across
// bond j+1 run as one batched Jacobi (every round launches the pair Grams
// and rotations of all gates still rotating, and each sweep ends in one
// read-back for all of them instead of one per gate), and the same again
// across bond j+2.  Every gate goes through the kernels, launch shapes,
// tolerances and sweeps it takes in gate_update, so the result is the same
// bit for bit; what changes is the number of launches and host round trips
// per layer, which bound the small-chi regime.
void fused_chunk(const std::vector<FusedJob>& jobs, tebd_mps* R, hipStream_t s) {
  const size_t cnt = jobs.size();
  std::vector<JacSvd> v(cnt);
  for (size_t i = 0; i < cnt; ++i) {
    const FusedJob& b = jobs[i];
    tebd_mps *M = b.M, *W = b.W;
    const int j = b.j, d = M->d;
    const int cl = M->chi[j], cr = M->chi[j + 3];
    W->ledger = M->wslots + j;
    theta_gate(M, W, j, b.G, s);
    JacSvd& x = v[i];
    x.W = W;
    x.in = SvdIn{W->psip.re, W->psip.im, (int64_t)d * d * cr, cl * d, d * d * cr, M->lam[j], d};
    x.lam_out = M->lam[j + 1];
    x.vhr = W->V1h.re;
    x.vhi = W->V1h.im;
    x.slot = 0;
    x.xbuf = W->psi;
  }
  jac_batch(R, v, s);
  std::vector<int> k1(cnt);
  for (size_t i = 0; i < cnt; ++i) {
    const FusedJob& b = jobs[i];
    tebd_mps *M = b.M, *W = b.W;
    const int j = b.j, d = M->d;
    const int cr = M->chi[j + 3];
    JacSvd& x = v[i];
    k1[i] = x.k;
    update_left_jacobi(M, W, j, x.in.m, x.in.n, k1[i], s);
    x.in = SvdIn{W->V1h.re, W->V1h.im, (int64_t)d * cr, k1[i] * d, d * cr, M->lam[j + 1], d};
    x.lam_out = M->lam[j + 2];
    x.vhr = M->Br[j + 2];
    x.vhi = M->Bi[j + 2];
    x.slot = 1;
    x.xbuf = W->X2;
  }
  jac_batch(R, v, s);
  for (size_t i = 0; i < cnt; ++i) {
    const FusedJob& b = jobs[i];
    update_middle_jacobi(b.M, b.W, b.j, v[i].in.m, v[i].in.n, v[i].k, s);
    b.M->chi[b.j + 1] = k1[i];
    b.M->chi[b.j + 2] = v[i].k;
  }
}

// The gates js of one layer of each handle Ms[h] (device gates G[h]), fused
// on the stream of Ms[0]: chunk c takes, from every handle, the gates
// c nw_h .. (c + 1) nw_h - 1 of its list, nw_h its number of workspaces.
void fused_run(const std::vector<tebd_mps*>& Ms, const std::vector<std::vector<int>>& js,
               const std::vector<std::vector<std::pair<double*, double*>>>& G) {
  tebd_mps* R = Ms[0]->workers[0];
  hipStream_t s = Ms[0]->stream;
  for (size_t c = 0;; ++c) {
    std::vector<FusedJob> jobs;
    for (size_t h = 0; h < Ms.size(); ++h) {
      const size_t nw = Ms[h]->workers.size();
      for (size_t w = 0; w < nw && c * nw + w < js[h].size(); ++w)
        jobs.push_back(FusedJob{Ms[h], Ms[h]->workers[w], js[h][c * nw + w], G[h][c * nw + w]});
    }
    if (jobs.empty()) return;
    fused_chunk(jobs, R, s);
  }
}

void fused_layer(tebd_mps* M, const std::vector<int>& js, const std::vector<std::pair<double*, double*>>& G) {
  fused_run({M}, {js}, {G});
}

}  // namespace

namespace {

// Adds the per-gate discarded weights of the layer to the ledger, in gate
// order (independent of how the gates were spread over workers).
void fold_ledger(tebd_mps* M) { accumulate_slots(M->wslots, M->L, M->ledger, M->stream); }

void run_gates(tebd_mps* M, const std::vector<int>& js, const std::vector<std::pair<double*, double*>>& G,
               bool parallel) {
  fill_zero(M->wslots, M->L, M->stream);
  const int nw = parallel ? std::min<int>((int)M->workers.size(), (int)js.size()) : 1;
  // A gate that fails leaves the layer half applied: the handle is marked
  // failed whatever the error, so that later calls refuse the state.
  if (parallel && M->opts.fuse) {
    try {
      fused_layer(M, js, G);
    } catch (...) {
      M->failed = true;
      throw;
    }
  } else if (nw <= 1) {
    tebd_mps* W = M->workers[0];
    try {
      for (size_t x = 0; x < js.size(); ++x) {
        W->ledger = M->wslots + js[x];
        update_gate(M, W, js[x], G[x]);
      }
    } catch (...) {
      M->failed = true;
      throw;
    }
  } else {
    // workers start after everything enqueued so far on the handle's stream
    hipEvent_t start;
    PTEBD_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    PTEBD_HIP(hipEventRecord(start, M->stream));
    for (int w = 1; w < nw; ++w) PTEBD_HIP(hipStreamWaitEvent(M->workers[w]->stream, start, 0));
    std::vector<std::exception_ptr> err(nw);
    Profiler* prof = active_profiler();
    auto work = [&](int w) {
      active_profiler() = prof;
      try {
        tebd_mps* W = M->workers[w];
        for (size_t x = w; x < js.size(); x += nw) {
          W->ledger = M->wslots + js[x];
          update_gate(M, W, js[x], G[x]);
        }
      } catch (...) {
        err[w] = std::current_exception();
      }
      active_profiler() = nullptr;
    };
    std::vector<std::thread> th;
    for (int w = 1; w < nw; ++w) th.emplace_back(work, w);
    work(0);
    active_profiler() = prof;
    for (auto& t : th) t.join();
    // the handle's stream continues after every worker
    for (int w = 1; w < nw; ++w) {
      hipEvent_t done;
      PTEBD_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
      PTEBD_HIP(hipEventRecord(done, M->workers[w]->stream));
      PTEBD_HIP(hipStreamWaitEvent(M->stream, done, 0));
      PTEBD_HIP(hipEventDestroy(done));
    }
    PTEBD_HIP(hipEventDestroy(start));
    for (int w = 0; w < nw; ++w)
      if (err[w]) {
        M->failed = true;
        std::rethrow_exception(err[w]);
      }
  }
  fold_ledger(M);
}

}  // namespace

// Left sites of the gates of one commuting group: j = group mod 3 for the
// three-site chain, K = group mod 2 for the super-site chain.
std::vector<int> group_gates(const tebd_mps* M, int group) {
  std::vector<int> js;
  if (M->super)
    for (int K = group; K + 1 < M->L; K += 2) js.push_back(K);
  else
    for (int j = group; j + 2 < M->L; j += 3) js.push_back(j);
  return js;
}

void layer(tebd_mps* M, int group, double tau) {
  std::vector<int> js;
  std::vector<std::pair<double*, double*>> G;
  for (int j : group_gates(M, group)) {
    js.push_back(j);
    G.push_back(device_gate(M, j, tau));
  }
  run_gates(M, js, G, true);
}

void layers_many(const std::vector<tebd_mps*>& Ms, int group, const std::vector<double>& taus) {
  const size_t n = Ms.size();
  hipStream_t s = Ms[0]->stream;
  std::vector<std::vector<int>> js(n);
  std::vector<std::vector<std::pair<double*, double*>>> G(n);
  for (size_t h = 0; h < n; ++h) {
    js[h] = group_gates(Ms[h], group);
    for (int j : js[h]) G[h].push_back(device_gate(Ms[h], j, taus[h]));
  }
  // stream s starts after the pending work of every handle, and every
  // handle's stream continues after s (so that freeing a handle, which
  // drains its own stream, also waits for the fused launches)
  auto join = [](hipStream_t from, hipStream_t to) {
    if (from == to) return;
    hipEvent_t e;
    PTEBD_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    PTEBD_HIP(hipEventRecord(e, from));
    PTEBD_HIP(hipStreamWaitEvent(to, e, 0));
    PTEBD_HIP(hipEventDestroy(e));
  };
  for (size_t h = 1; h < n; ++h) join(Ms[h]->stream, s);
  for (tebd_mps* M : Ms) fill_zero(M->wslots, M->L, s);
  try {
    fused_run(Ms, js, G);
  } catch (...) {
    // every handle of the batch is left half applied; the launches already
    // queued still touch their buffers, so they drain before anyone frees them
    for (tebd_mps* M : Ms) M->failed = true;
    (void)hipStreamSynchronize(s);
    throw;
  }
  for (tebd_mps* M : Ms) accumulate_slots(M->wslots, M->L, M->ledger, s);
  for (size_t h = 1; h < n; ++h) join(s, Ms[h]->stream);
}

void canonicalize(tebd_mps* M) {
  // identity gates swept left to right: each exposes the exact Schmidt
  // decomposition across its two inner bonds given the left Lambda
  std::vector<int> js;
  std::vector<std::pair<double*, double*>> G;
  for (int j = 0; j + (M->super ? 1 : 2) < M->L; ++j) {
    js.push_back(j);
    G.push_back(device_gate(M, j, 0.0));
  }
  run_gates(M, js, G, false);
}

void sweep_stats(const tebd_mps* M, int64_t* last, int64_t* total) {
  *last = 0;
  *total = 0;
  for (const tebd_mps* W : M->workers) {
    *last = std::max<int64_t>(*last, W->last_sweeps);
    *total += W->total_sweeps;
  }
}

void trunc_stats(const tebd_mps* M, int64_t* counts) {
  for (int i = 0; i < 4; ++i) counts[i] = 0;
  for (const tebd_mps* W : M->workers)
    for (int i = 0; i < 4; ++i) counts[i] += W->rule_counts[i];
}

void prepare_gates(tebd_mps* M, int group, double tau) {
  for (int j : group_gates(M, group)) (void)device_gate(M, j, tau);
}

namespace {

// Physical n, <b+_i b_{i+1}> and <b+_i b_{i+2}> of a super-site chain: the
// densities and the correlator inside a super site are local to it; the
// correlators across super sites K, K+1 close an environment carrying the
// creation operator on K with the annihilation operator on K+1.
void measure_super(tebd_mps* M, double* n_out, double* cnn, double* cnnn) {
  hipStream_t s = M->stream;
  const int Ls = M->L, D = M->d, d = M->pd, L = M->phys_L;
  PTEBD_HIP(hipMemcpyAsync(M->d_chi, M->chi.data(), sizeof(int) * (Ls + 1), hipMemcpyHostToDevice, s));
  double* loc = M->meas;               // 4 per super site
  double* c_odd = M->meas + 4 * Ls;    // <b+_{2K+1} b_{2K+2}>
  double* d_even = M->meas + 6 * Ls;   // <b+_{2K} b_{2K+2}>
  double* d_odd = M->meas + 8 * Ls;    // <b+_{2K+1} b_{2K+3}>
  supersite_local(M->d_br, M->d_bi, M->d_lam, M->d_chi, M->d_chi + 1, Ls, d, loc, s);
  const bool want = cnn || cnnn;
  for (int K = 0; want && K + 1 < Ls; ++K) {
    const int cl = M->chi[K], cr = M->chi[K + 1], cr2 = M->chi[K + 2];
    // creation operator on the second (mode 2) then on the first (mode 1) site of K
    for (int mode1 = 2; mode1 >= 1; --mode1) {
      const int shift1 = mode1 == 1 ? d : 1;
      op_kscale(M->lam[K], cl, D, d, shift1, mode1, M->ks, s);
      {  // E = sum Lambda^2 sqrt(level) B(a, s, .)^+ B(a, s - shift, .)
        ZGemmArgs g;
        g.m = cr; g.n = cr; g.k = cl * D - shift1;
        g.ar = M->Br[K] + (int64_t)shift1 * cr; g.ai = M->Bi[K] + (int64_t)shift1 * cr; g.lda = cr; g.transA = 1;
        g.br = M->Br[K]; g.bi = M->Bi[K]; g.ldb = cr;
        g.cr = M->E.re; g.ci = M->E.im; g.ldc = cr;
        g.k_scale = M->ks;
        g.tag = "measure";
        zgemm(g, 0, s);
      }
      {  // F = E B_{K+1}
        ZGemmArgs g;
        g.m = cr; g.n = D * cr2; g.k = cr;
        g.ar = M->E.re; g.ai = M->E.im; g.lda = cr;
        g.br = M->Br[K + 1]; g.bi = M->Bi[K + 1]; g.ldb = (int64_t)D * cr2;
        g.cr = M->F.re; g.ci = M->F.im; g.ldc = (int64_t)D * cr2;
        g.tag = "measure";
        zgemm(g, 0, s);
      }
      if (mode1 == 2) {
        // b+_{2K+1} b_{2K+2} (first site of K+1) and b+_{2K+1} b_{2K+3} (second site)
        close_op(M->Br[K + 1], M->Bi[K + 1], M->F.re, M->F.im, cr, D, cr2, d, d, 1, c_odd + 2 * K, M->hop_part, s);
        close_op(M->Br[K + 1], M->Bi[K + 1], M->F.re, M->F.im, cr, D, cr2, d, 1, 2, d_odd + 2 * K, M->hop_part, s);
      } else {
        // b+_{2K} b_{2K+2}
        close_op(M->Br[K + 1], M->Bi[K + 1], M->F.re, M->F.im, cr, D, cr2, d, d, 1, d_even + 2 * K, M->hop_part, s);
      }
    }
  }
  std::vector<double> h(10 * (size_t)Ls);
  PTEBD_HIP(hipMemcpyAsync(h.data(), M->meas, sizeof(double) * 10 * Ls, hipMemcpyDeviceToHost, s));
  PTEBD_HIP(hipStreamSynchronize(s));
  for (int K = 0; K < Ls; ++K) {
    if (n_out) {
      n_out[2 * K] = h[4 * K];
      n_out[2 * K + 1] = h[4 * K + 1];
    }
    if (cnn) {
      cnn[2 * (2 * K)] = h[4 * K + 2];
      cnn[2 * (2 * K) + 1] = h[4 * K + 3];
      if (K + 1 < Ls) {
        cnn[2 * (2 * K + 1)] = h[4 * Ls + 2 * K];
        cnn[2 * (2 * K + 1) + 1] = h[4 * Ls + 2 * K + 1];
      }
    }
    if (cnnn && K + 1 < Ls) {
      cnnn[2 * (2 * K)] = h[6 * Ls + 2 * K];
      cnnn[2 * (2 * K) + 1] = h[6 * Ls + 2 * K + 1];
      cnnn[2 * (2 * K + 1)] = h[8 * Ls + 2 * K];
      cnnn[2 * (2 * K + 1) + 1] = h[8 * Ls + 2 * K + 1];
    }
  }
  (void)L;
}

}  // namespace

void measure(tebd_mps* M, double* n_out, double* cnn, double* cnnn) {
  if (M->super) {
    measure_super(M, n_out, cnn, cnnn);
    return;
  }
  hipStream_t s = M->stream;
  const int L = M->L, d = M->d;
  PTEBD_HIP(hipMemcpyAsync(M->d_chi, M->chi.data(), sizeof(int) * (L + 1), hipMemcpyHostToDevice, s));
  double* dn = M->meas;
  double* dc = M->meas + L;
  double* dd = M->meas + 3 * L;
  site_densities(M->d_br, M->d_bi, M->d_lam, M->d_chi, M->d_chi + 1, L, d, dn, s);
  const bool want_hops = cnn || cnnn;
  for (int i = 0; want_hops && i + 1 < L; ++i) {
    const int cl = M->chi[i], cr = M->chi[i + 1], cr2 = M->chi[i + 2];
    op_kscale(M->lam[i], cl, d, d, 1, 0, M->ks, s);
    {  // E = sum Lambda^2 sqrt(s) B(a,s,.)^+ B(a,s-1,.)
      ZGemmArgs g;
      g.m = cr; g.n = cr; g.k = cl * d - 1;
      g.ar = M->Br[i] + cr; g.ai = M->Bi[i] + cr; g.lda = cr; g.transA = 1;
      g.br = M->Br[i]; g.bi = M->Bi[i]; g.ldb = cr;
      g.cr = M->E.re; g.ci = M->E.im; g.ldc = cr;
      g.k_scale = M->ks;
      g.tag = "measure";
      zgemm(g, 0, s);
    }
    {  // F = E B_{i+1}
      ZGemmArgs g;
      g.m = cr; g.n = d * cr2; g.k = cr;
      g.ar = M->E.re; g.ai = M->E.im; g.lda = cr;
      g.br = M->Br[i + 1]; g.bi = M->Bi[i + 1]; g.ldb = (int64_t)d * cr2;
      g.cr = M->F.re; g.ci = M->F.im; g.ldc = (int64_t)d * cr2;
      g.tag = "measure";
      zgemm(g, 0, s);
    }
    close_op(M->Br[i + 1], M->Bi[i + 1], M->F.re, M->F.im, cr, d, cr2, d, 1, 0, dc + 2 * i, M->hop_part, s);
    if (i + 2 < L) {
      const int cr3 = M->chi[i + 3];
      {  // F2 = B_{i+1}^+ F   (rows (y, s) contracted)
        ZGemmArgs g;
        g.m = cr2; g.n = cr2; g.k = cr * d;
        g.ar = M->Br[i + 1]; g.ai = M->Bi[i + 1]; g.lda = cr2; g.transA = 1;
        g.br = M->F.re; g.bi = M->F.im; g.ldb = cr2;
        g.cr = M->F2.re; g.ci = M->F2.im; g.ldc = cr2;
        g.tag = "measure";
        zgemm(g, 0, s);
      }
      {  // F3 = F2 B_{i+2}
        ZGemmArgs g;
        g.m = cr2; g.n = d * cr3; g.k = cr2;
        g.ar = M->F2.re; g.ai = M->F2.im; g.lda = cr2;
        g.br = M->Br[i + 2]; g.bi = M->Bi[i + 2]; g.ldb = (int64_t)d * cr3;
        g.cr = M->F3.re; g.ci = M->F3.im; g.ldc = (int64_t)d * cr3;
        g.tag = "measure";
        zgemm(g, 0, s);
      }
      close_op(M->Br[i + 2], M->Bi[i + 2], M->F3.re, M->F3.im, cr2, d, cr3, d, 1, 0, dd + 2 * i, M->hop_part, s);
    }
  }
  std::vector<double> h(5 * (size_t)L);
  PTEBD_HIP(hipMemcpyAsync(h.data(), M->meas, sizeof(double) * 5 * L, hipMemcpyDeviceToHost, s));
  PTEBD_HIP(hipStreamSynchronize(s));
  if (n_out) std::memcpy(n_out, h.data(), sizeof(double) * L);
  if (cnn && L >= 2) std::memcpy(cnn, h.data() + L, sizeof(double) * 2 * (L - 1));
  if (cnnn && L >= 3) std::memcpy(cnnn, h.data() + 3 * L, sizeof(double) * 2 * (L - 2));
}

}  // namespace ptebd
