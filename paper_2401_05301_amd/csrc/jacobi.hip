// One-sided block Jacobi (Hestenes) SVD engine, FP64, for gfx950.
//
// The rows of X (r x c) are made mutually orthogonal by unitary mixing of
// pairs of 16-row blocks.  One sweep visits every block pair once, in nb-1
// rounds of nb/2 disjoint pairs (round-robin "circle" ordering).  For a pair
// (I, J) with rows R = I u J (32 rows):
//   1. C = X_R X_R^+ (32 x 32 Hermitian) is accumulated with FP64 MFMA over
//      column splits (jac_gram), then summed in a fixed order;
//   2. if some |C_pq| exceeds max(tol_rel sqrt(C_pp C_qq), tol_abs), C is
//      diagonalised in LDS by cyclic two-sided Jacobi rotations, Q^+ C Q = D;
//   3. X_R <- Q^+ X_R (and W_R <- Q^+ W_R) with FP64 MFMA (jac_rotate).
// At convergence the row norms of X are the singular values (or, when X is a
// Gram matrix G, its eigenvalues) and W holds the accumulated unitary.
#include <mutex>

#include "kernels.hpp"
#include "profile.hpp"

namespace ptebd {

namespace {

constexpr int JB = 16;       // rows per block
constexpr int PR = 2 * JB;   // rows per pair

__device__ __forceinline__ f64x4 mfma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of accumulator element e of a 16x16 FP64 MFMA result held by `lane`
// (the column is lane % 16).
__device__ __forceinline__ int acc_row(int lane, int e) { return (lane >> 4) + 4 * e; }

// Block pair of round `t` (0 <= t < nb-1), pair slot `p` (0 <= p < nb/2).
__device__ __forceinline__ void round_pair(int nb, int t, int p, int& I, int& J) {
  auto pos = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + t) % (nb - 1); };
  int a = pos(p), b = pos(nb - 1 - p);
  I = a < b ? a : b;
  J = a < b ? b : a;
}

__device__ __forceinline__ int pair_row(int I, int J, int k) { return k < JB ? I * JB + k : J * JB + (k - JB); }

// ------------------------------------------------------------ partial Grams
// One work-group per (pair, column split); part layout per (pair, split):
// [tile aa, ab, bb][re, im][16*16]
__device__ __forceinline__ void jac_gram_body(const JacobiArgs& a, int round, int pair, int split,
                                              double (*red)[3][2][256]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int I, J;
  round_pair(a.nb, round, pair, I, J);
  const int chunk = ((a.c + a.nsplit - 1) / a.nsplit + 15) / 16 * 16;
  const int cb = split * chunk;
  const int ce = min(a.c, cb + chunk);
  const int ra = I * JB + (lane & 15), rb = J * JB + (lane & 15);
  const bool va = ra < a.r, vb = rb < a.r;
  const double* xar = a.xr + (int64_t)ra * a.ldx;
  const double* xai = a.xi + (int64_t)ra * a.ldx;
  const double* xbr = a.xr + (int64_t)rb * a.ldx;
  const double* xbi = a.xi + (int64_t)rb * a.ldx;

  f64x4 g[3][2];
#pragma unroll
  for (int t = 0; t < 3; ++t) g[t][0] = g[t][1] = f64x4{0, 0, 0, 0};

  // each wave walks 16-column groups; lane holds 4 consecutive columns of its row
  for (int c0 = cb + wave * 16; c0 < ce; c0 += 64) {
    const int cc = c0 + (lane >> 4) * 4;
    double ar[4], ai[4], br[4], bi[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int col = cc + e;
      const bool ok = col < ce;
      ar[e] = (va && ok) ? xar[col] : 0.0;
      ai[e] = (va && ok) ? xai[col] : 0.0;
      br[e] = (vb && ok) ? xbr[col] : 0.0;
      bi[e] = (vb && ok) ? xbi[col] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      // G_xy[p,q] = sum_k x_p,k conj(y_q,k): re = xr yr + xi yi, im = xi yr - xr yi
      g[0][0] = mfma(ar[e], ar[e], g[0][0]);
      g[0][0] = mfma(ai[e], ai[e], g[0][0]);
      g[0][1] = mfma(ai[e], ar[e], g[0][1]);
      g[0][1] = mfma(-ar[e], ai[e], g[0][1]);
      g[1][0] = mfma(ar[e], br[e], g[1][0]);
      g[1][0] = mfma(ai[e], bi[e], g[1][0]);
      g[1][1] = mfma(ai[e], br[e], g[1][1]);
      g[1][1] = mfma(-ar[e], bi[e], g[1][1]);
      g[2][0] = mfma(br[e], br[e], g[2][0]);
      g[2][0] = mfma(bi[e], bi[e], g[2][0]);
      g[2][1] = mfma(bi[e], br[e], g[2][1]);
      g[2][1] = mfma(-br[e], bi[e], g[2][1]);
    }
  }
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int ri = 0; ri < 2; ++ri)
#pragma unroll
      for (int e = 0; e < 4; ++e) red[wave][t][ri][acc_row(lane, e) * 16 + (lane & 15)] = g[t][ri][e];
  __syncthreads();
  double* out = a.part + ((int64_t)pair * a.nsplit + split) * 1536;
  for (int idx = threadIdx.x; idx < 1536; idx += 256) {
    const int t = idx / 512, ri = (idx / 256) & 1, el = idx & 255;
    out[idx] = ((red[0][t][ri][el] + red[1][t][ri][el]) + red[2][t][ri][el]) + red[3][t][ri][el];
  }
}

// grid (nb/2, nsplit)
__global__ __launch_bounds__(256) void jac_gram(JacobiArgs a, int round) {
  __shared__ double red[4][3][2][256];
  jac_gram_body(a, round, blockIdx.x, blockIdx.y, red);
}

// ------------------------------------------------- pair eigensolve + update
struct RotLds {
  double Cr[PR][PR + 1], Ci[PR][PR + 1], Qr[PR][PR + 1], Qi[PR][PR + 1];
  double rot[16][4];
};

// One work-group per (pair, column chunk of the update).
__device__ __forceinline__ void jac_rotate_body(const JacobiArgs& a, int round, int pair, int chunk_id, RotLds& L) {
  auto& Cr = L.Cr;
  auto& Ci = L.Ci;
  auto& Qr = L.Qr;
  auto& Qi = L.Qi;
  auto& rot = L.rot;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int I, J;
  round_pair(a.nb, round, pair, I, J);

  // 1. sum the partial Grams in a fixed order
  const double* part = a.part + (int64_t)pair * a.nsplit * 1536;
  for (int idx = tid; idx < PR * PR; idx += 256) {
    const int p = idx / PR, q = idx % PR;
    int t, pp, qq;
    bool cj = false;
    if (p < JB && q < JB) { t = 0; pp = p; qq = q; }
    else if (p < JB) { t = 1; pp = p; qq = q - JB; }
    else if (q < JB) { t = 1; pp = q; qq = p - JB; cj = true; }
    else { t = 2; pp = p - JB; qq = q - JB; }
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < a.nsplit; ++s) {
      sr += part[s * 1536 + t * 512 + pp * 16 + qq];
      si += part[s * 1536 + t * 512 + 256 + pp * 16 + qq];
    }
    Cr[p][q] = sr;
    Ci[p][q] = cj ? -si : si;
    Qr[p][q] = (p == q) ? 1.0 : 0.0;
    Qi[p][q] = 0.0;
  }
  __syncthreads();

  // 2. outer convergence test on this pair.  A row whose squared norm is at
  // the rounding level of the whole matrix is treated as zero: rotating it
  // only reshuffles noise (and two exactly parallel rows would otherwise
  // leave a parallel residual forever).
  const double tiny2 = *a.tiny2;
  int need = 0;
  for (int idx = tid; idx < PR * PR; idx += 256) {
    const int p = idx / PR, q = idx % PR;
    if (p < q) {
      const double app = Cr[p][p], aqq = Cr[q][q];
      if (app <= tiny2 || aqq <= tiny2) continue;
      const double c = hypot(Cr[p][q], Ci[p][q]);
      if (c > fmax(a.tol_rel * sqrt(app) * sqrt(aqq), a.tol_abs)) need = 1;
    }
  }
  if (!__syncthreads_or(need)) return;
  if (chunk_id == 0 && tid == 0) atomicAdd(a.rotated, 1u);

  // 3. cyclic Jacobi on the 32 x 32 Hermitian pair matrix
  for (int sweep = 0; sweep < 12; ++sweep) {
    int changed = 0;
    for (int st = 0; st < PR - 1; ++st) {
      if (tid < 16) {
        auto pos = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + st) % (PR - 1); };
        const int p0 = pos(tid), q0 = pos(PR - 1 - tid);
        const int p = min(p0, q0), q = max(p0, q0);
        const double app = Cr[p][p], aqq = Cr[q][q];
        const double cre = Cr[p][q], cim = Ci[p][q];
        const double c = hypot(cre, cim);
        double cs = 1.0, sn = 0.0, er = 1.0, ei = 0.0;
        // the inner solve goes four times below the outer test so that a
        // diagonalised pair passes that test on the next sweep
        if (app > tiny2 && aqq > tiny2 &&
            c > fmax(0.25 * a.tol_rel * sqrt(app) * sqrt(aqq), 0.25 * a.tol_abs)) {
          const double tau = (aqq - app) / (2.0 * c);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          cs = 1.0 / sqrt(1.0 + t * t);
          sn = t * cs;
          er = cre / c;   // e^{-i phi} = conj(c) / |c|
          ei = -cim / c;
          changed = 1;
        }
        rot[tid][0] = cs; rot[tid][1] = sn; rot[tid][2] = er; rot[tid][3] = ei;
      }
      __syncthreads();
      // rows: C <- J^+ C   (row p: cs rp - sn e^{i phi} rq ; row q: sn rp + cs e^{i phi} rq)
      for (int it = tid; it < 16 * PR; it += 256) {
        const int k = it / PR, col = it % PR;
        auto pos = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + st) % (PR - 1); };
        const int p0 = pos(k), q0 = pos(PR - 1 - k);
        const int p = min(p0, q0), q = max(p0, q0);
        const double cs = rot[k][0], sn = rot[k][1], er = rot[k][2], ei = -rot[k][3];  // e^{+i phi}
        if (sn == 0.0) continue;
        const double pr_ = Cr[p][col], pi_ = Ci[p][col], qr_ = Cr[q][col], qi_ = Ci[q][col];
        const double tr_ = er * qr_ - ei * qi_, ti_ = er * qi_ + ei * qr_;
        Cr[p][col] = cs * pr_ - sn * tr_;
        Ci[p][col] = cs * pi_ - sn * ti_;
        Cr[q][col] = sn * pr_ + cs * tr_;
        Ci[q][col] = sn * pi_ + cs * ti_;
      }
      __syncthreads();
      // columns: C <- C J, Q <- Q J  (col p: cs cp - sn e^{-i phi} cq ; col q: sn cp + cs e^{-i phi} cq)
      for (int it = tid; it < 16 * PR; it += 256) {
        const int k = it / PR, row = it % PR;
        auto pos = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + st) % (PR - 1); };
        const int p0 = pos(k), q0 = pos(PR - 1 - k);
        const int p = min(p0, q0), q = max(p0, q0);
        const double cs = rot[k][0], sn = rot[k][1], er = rot[k][2], ei = rot[k][3];
        if (sn == 0.0) continue;
        {
          const double pr_ = Cr[row][p], pi_ = Ci[row][p], qr_ = Cr[row][q], qi_ = Ci[row][q];
          const double tr_ = er * qr_ - ei * qi_, ti_ = er * qi_ + ei * qr_;
          Cr[row][p] = cs * pr_ - sn * tr_;
          Ci[row][p] = cs * pi_ - sn * ti_;
          Cr[row][q] = sn * pr_ + cs * tr_;
          Ci[row][q] = sn * pi_ + cs * ti_;
        }
        {
          const double pr_ = Qr[row][p], pi_ = Qi[row][p], qr_ = Qr[row][q], qi_ = Qi[row][q];
          const double tr_ = er * qr_ - ei * qi_, ti_ = er * qi_ + ei * qr_;
          Qr[row][p] = cs * pr_ - sn * tr_;
          Qi[row][p] = cs * pi_ - sn * ti_;
          Qr[row][q] = sn * pr_ + cs * tr_;
          Qi[row][q] = sn * pi_ + cs * ti_;
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(changed)) break;
  }

  // 4. X_R <- Q^+ X_R on this work-group's column chunk (X columns, then W columns)
  // A operand Q^+(p, k) = conj(Q(k, p)); lane: p = lane%16 (+16 tile), k = 4*ks + lane/16
  double qar[2][8], qai[2][8];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int p = t * 16 + (lane & 15), k = 4 * ks + (lane >> 4);
      qar[t][ks] = Qr[k][p];
      qai[t][ks] = -Qi[k][p];
    }
  const int total = a.c + (a.wr ? a.r : 0);
  const int cb = chunk_id * a.ucols;
  const int ce = min(total, cb + a.ucols);
  for (int j0 = cb + wave * 16; j0 < ce; j0 += 64) {
    const int j = j0 + (lane & 15);
    const bool inw = j >= a.c;
    const bool okc = j < ce;
    double* baser = inw ? a.wr : a.xr;
    double* basei = inw ? a.wi : a.xi;
    const int64_t ld = inw ? a.ldw : a.ldx;
    const int col = inw ? j - a.c : j;
    double xr[8], xi[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int k = 4 * ks + (lane >> 4);
      const int row = pair_row(I, J, k);
      const bool ok = okc && row < a.r;
      xr[ks] = ok ? baser[(int64_t)row * ld + col] : 0.0;
      xi[ks] = ok ? basei[(int64_t)row * ld + col] : 0.0;
    }
    f64x4 orr[2], oii[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      orr[t] = f64x4{0, 0, 0, 0};
      oii[t] = f64x4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        orr[t] = mfma(qar[t][ks], xr[ks], orr[t]);
        orr[t] = mfma(-qai[t][ks], xi[ks], orr[t]);
        oii[t] = mfma(qar[t][ks], xi[ks], oii[t]);
        oii[t] = mfma(qai[t][ks], xr[ks], oii[t]);
      }
    }
    // the 16 columns of this slab may straddle the X / W boundary: each lane
    // stores its own column, so recompute the destination per output element
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = t * 16 + acc_row(lane, e);
        const int row = pair_row(I, J, k);
        if (okc && row < a.r) {
          baser[(int64_t)row * ld + col] = orr[t][e];
          basei[(int64_t)row * ld + col] = oii[t][e];
        }
      }
  }
}

// grid (nb/2, nuchunks)
__global__ __launch_bounds__(256) void jac_rotate(JacobiArgs a, int round) {
  __shared__ RotLds L;
  jac_rotate_body(a, round, blockIdx.x, blockIdx.y, L);
}

// Batched form over independent matrices (one JacobiArgs each in the device
// table tab): first[i] is the first work-group of matrix i (first[count] the
// total); a matrix takes part while active[i] != 0 and round < nb_i - 1.

__global__ __launch_bounds__(256) void jac_gram_batched(const JacobiArgs* tab, const int64_t* first, int count,
                                                        const int* active, int round) {
  __shared__ double red[4][3][2][256];
  const int i = batch_owner(first, count, blockIdx.x);
  const JacobiArgs a = tab[i];
  if (!active[i] || round >= a.nb - 1) return;
  const int local = (int)(blockIdx.x - first[i]);
  jac_gram_body(a, round, local / a.nsplit, local % a.nsplit, red);
}

__global__ __launch_bounds__(256) void jac_rotate_batched(const JacobiArgs* tab, const int64_t* first, int count,
                                                          const int* active, int round) {
  __shared__ RotLds L;
  const int i = batch_owner(first, count, blockIdx.x);
  const JacobiArgs a = tab[i];
  if (!active[i] || round >= a.nb - 1) return;
  const int local = (int)(blockIdx.x - first[i]);
  jac_rotate_body(a, round, local / a.nuchunks, local % a.nuchunks, L);
}

// One wave per row: the 2-norm of row `row` of the r x c matrix x.
__device__ __forceinline__ void row_norm_body(const double* xr, const double* xi, int64_t ldx, int r, int c,
                                              double* norms) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= r) return;
  const double* pr = xr + (int64_t)row * ldx;
  const double* pi = xi + (int64_t)row * ldx;
  double s = 0.0;
  for (int j = lane; j < c; j += 64) s += pr[j] * pr[j] + pi[j] * pi[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) norms[row] = sqrt(s);
}

__global__ __launch_bounds__(256) void row_norms_kernel(const double* xr, const double* xi, int64_t ldx,
                                                        int r, int c, double* norms) {
  row_norm_body(xr, xi, ldx, r, c, norms);
}

// matrix blockIdx.y of the batch
__global__ __launch_bounds__(256) void fused_row_norms_kernel(const FusedSvdArgs* tab) {
  const FusedSvdArgs& a = tab[blockIdx.y];
  row_norm_body(a.yr, a.yi, a.c, a.r, a.c, a.norms);
}

// Single work-group: bitonic sort (descending value, ascending index on ties),
// then the truncation rule, sequentially in FP64 by one thread.  key and idx
// hold npow2 entries of LDS; s_k and s_nrm are LDS scalars.
__device__ __forceinline__ void select_body(const double* vals, int r, int npow2, int is_gram, int chi_max,
                                            double w_max, double eps, double* lam_out, int* perm, double* inv_sig,
                                            int* info_i, double* info_d, double* ledger, const double* extra_tail,
                                            double* key, int* idx, int& s_k, double& s_nrm) {
  for (int i = threadIdx.x; i < npow2; i += 256) {
    if (i < r) {
      const double v = vals[i];
      key[i] = is_gram ? sqrt(fmax(v, 0.0)) : v;
      idx[i] = i;
    } else {
      key[i] = -1.0;
      idx[i] = 0x7fffffff;
    }
  }
  __syncthreads();
  // "before": a precedes b in the final order
  for (int size = 2; size <= npow2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < npow2; i += 256) {
        const int l = i ^ stride;
        if (l > i) {
          const bool desc = (i & size) == 0;
          const double ki = key[i], kl = key[l];
          const int ii = idx[i], il = idx[l];
          const bool l_first = (kl > ki) || (kl == ki && il < ii);
          if (l_first == desc) {
            key[i] = kl; key[l] = ki;
            idx[i] = il; idx[l] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    const double extra = extra_tail ? fmax(extra_tail[0], 0.0) : 0.0;
    double total = extra;
    for (int i = 0; i < r; ++i) total += key[i] * key[i];
    int k, rule = 3;
    double tail_k = 0.0;
    if (total <= 0.0) {
      k = 1;
      tail_k = 0.0;
    } else {
      // k_w: smallest k with sum_{i>=k} s_i^2 <= w_max * total
      double acc = extra;
      int kw = r;
      // tails accumulated from the smallest value upwards
      // (walk down while the tail stays within the tolerance)
      for (int i = r - 1; i >= 0; --i) {
        const double nxt = acc + key[i] * key[i];
        if (nxt <= w_max * total) {
          acc = nxt;
          kw = i;
        } else {
          break;
        }
      }
      int ke = 0;
      const double thr = eps * key[0];
      for (int i = 0; i < r; ++i)
        if (key[i] > thr) ke = i + 1;
      k = min(min(chi_max, kw), ke);
      if (k < 1) k = 1;
      if (k > r) k = r;
      // the part of the rule that set k (precedence chi_max, k_w, k_eps)
      if (k < r) rule = (k == chi_max) ? 0 : (k == kw) ? 1 : (k == ke) ? 2 : 3;
      tail_k = extra;
      for (int i = r - 1; i >= k; --i) tail_k += key[i] * key[i];
    }
    double kept = 0.0;
    for (int i = 0; i < k; ++i) kept += key[i] * key[i];
    double nrm = sqrt(kept);
    if (!(nrm > 0.0)) nrm = 1.0;
    const double w = total > 0.0 ? tail_k / total : 0.0;
    info_i[0] = k;
    info_i[4] = rule;
    info_d[0] = nrm;
    info_d[13] = key[0] > 0.0 ? key[k - 1] / key[0] : 1.0;   // smallest kept over largest value
    info_d[1] = w;
    *ledger += w;
    s_k = k;
    s_nrm = nrm;
  }
  __syncthreads();
  const int k = s_k;
  const double nrm = s_nrm;
  for (int i = threadIdx.x; i < k; i += 256) {
    lam_out[i] = key[i] / nrm;
    perm[i] = idx[i];
    inv_sig[i] = key[i] > 0.0 ? 1.0 / key[i] : 0.0;
  }
}

__global__ __launch_bounds__(256) void select_kernel(const double* vals, int r, int npow2, int is_gram,
                                                     int chi_max, double w_max, double eps, double* lam_out,
                                                     int* perm, double* inv_sig, int* info_i, double* info_d,
                                                     double* ledger, const double* extra_tail) {
  extern __shared__ unsigned char smem[];
  __shared__ int s_k;
  __shared__ double s_nrm;
  double* key = reinterpret_cast<double*>(smem);
  select_body(vals, r, npow2, is_gram, chi_max, w_max, eps, lam_out, perm, inv_sig, info_i, info_d, ledger,
              extra_tail, key, reinterpret_cast<int*>(key + npow2), s_k, s_nrm);
}

// matrix blockIdx.x of the batch; LDS sized for the largest npow2
__global__ __launch_bounds__(256) void fused_select_kernel(const FusedSvdArgs* tab) {
  extern __shared__ unsigned char smem[];
  __shared__ int s_k;
  __shared__ double s_nrm;
  const FusedSvdArgs& a = tab[blockIdx.x];
  double* key = reinterpret_cast<double*>(smem);
  select_body(a.norms, a.r, a.npow2, a.is_gram, a.chi_max, a.w_max, a.eps, a.lam_out, a.perm, a.inv_sig, a.info_i,
              a.info_d, a.ledger, a.extra_tail, key, reinterpret_cast<int*>(key + a.npow2), s_k, s_nrm);
  if (threadIdx.x == 0) {
    a.kout[0] = s_k;
    a.kout[1] = a.info_i[4];
  }
}

__device__ __forceinline__ void negligible_body(const double* norms, int r, double* out, double* sh) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < r; i += 256) acc += norms[i] * norms[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double u4 = 4.0 * 1.1102230246251565e-16;
    out[0] = u4 * u4 * sh[0];
  }
}

__global__ __launch_bounds__(256) void negligible_kernel(const double* norms, int r, double* out) {
  __shared__ double sh[256];
  negligible_body(norms, r, out, sh);
}

// blockIdx.y == 0: negligible_norm2 of matrix blockIdx.z; blockIdx.y > 0:
// row blockIdx.y - 1 of the identity in its vectors (transposed matrices)
__global__ __launch_bounds__(256) void fused_prologue_kernel(const FusedSvdArgs* tab, double* out) {
  __shared__ double sh[256];
  const FusedSvdArgs& a = tab[blockIdx.z];
  if (blockIdx.y == 0) {
    if (blockIdx.x == 0) negligible_body(a.norms, a.r, out + blockIdx.z, sh);
    return;
  }
  const int i = (int)blockIdx.y - 1;
  if (!a.transpose || i >= a.r) return;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < a.r; j += gridDim.x * blockDim.x) {
    a.wr[(int64_t)i * a.ldw + j] = (i == j) ? 1.0 : 0.0;
    a.wi[(int64_t)i * a.ldw + j] = 0.0;
  }
}

__device__ __forceinline__ void gather_body(const double* sr, const double* si, int64_t lds, const int* perm,
                                            const double* scale, int k, int c, double* dr, double* di,
                                            int64_t ldd) {
  const int i = blockIdx.y;
  if (i >= k) return;
  const int src = perm[i];
  const double s = scale ? scale[i] : 1.0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < c; j += gridDim.x * blockDim.x) {
    dr[(int64_t)i * ldd + j] = sr[(int64_t)src * lds + j] * s;
    di[(int64_t)i * ldd + j] = si[(int64_t)src * lds + j] * s;
  }
}

__global__ void gather_kernel(const double* sr, const double* si, int64_t lds, const int* perm,
                              const double* scale, int k, int c, double* dr, double* di, int64_t ldd) {
  gather_body(sr, si, lds, perm, scale, k, c, dr, di, ldd);
}

// matrix blockIdx.z of the batch, k from its kout
__global__ void fused_gather_kernel(const FusedSvdArgs* tab) {
  const FusedSvdArgs& a = tab[blockIdx.z];
  gather_body(a.gr, a.gi, a.ldg, a.perm, a.gscale ? a.inv_sig : nullptr, a.kout[0], a.gc, a.dr, a.di, a.ldd);
}

}  // namespace

void jacobi_round(const JacobiArgs& a, int round, hipStream_t s) {
  dim3 g1(a.nb / 2, a.nsplit);
  {
    ProfScope ps(K_JAC_GRAM, 0.0, s);
    jac_gram<<<g1, 256, 0, s>>>(a, round);
    PTEBD_LAUNCH_CHECK();
  }
  dim3 g2(a.nb / 2, a.nuchunks);
  {
    ProfScope ps(K_JAC_ROTATE, 0.0, s);
    jac_rotate<<<g2, 256, 0, s>>>(a, round);
    PTEBD_LAUNCH_CHECK();
  }
}

void jacobi_round_batched(const JacobiArgs* tab, const int64_t* gram_first, int64_t gram_total,
                          const int64_t* rot_first, int64_t rot_total, int count, const int* active, int round,
                          hipStream_t s) {
  {
    ProfScope ps(K_JAC_GRAM, 0.0, s);
    jac_gram_batched<<<(unsigned)gram_total, 256, 0, s>>>(tab, gram_first, count, active, round);
    PTEBD_LAUNCH_CHECK();
  }
  {
    ProfScope ps(K_JAC_ROTATE, 0.0, s);
    jac_rotate_batched<<<(unsigned)rot_total, 256, 0, s>>>(tab, rot_first, count, active, round);
    PTEBD_LAUNCH_CHECK();
  }
}

void negligible_norm2(const double* norms, int r, double* out, hipStream_t s) {
  negligible_kernel<<<1, 256, 0, s>>>(norms, r, out);
  PTEBD_LAUNCH_CHECK();
}

void row_norms(const double* xr, const double* xi, int64_t ldx, int r, int c, double* norms, hipStream_t s) {
  row_norms_kernel<<<ceil_div(r, 4), 256, 0, s>>>(xr, xi, ldx, r, c, norms);
  PTEBD_LAUNCH_CHECK();
}

void select_truncate(const double* vals, int r, int is_gram, int chi_max, double w_max, double eps,
                     double* lam_out, int* perm, double* inv_sig, int* info_i, double* info_d, double* ledger,
                     const double* extra_tail, hipStream_t s) {
  int np2 = 1;
  while (np2 < r) np2 <<= 1;
  const size_t shm = (size_t)np2 * (sizeof(double) + sizeof(int));
  constexpr size_t kMaxShm = 96 * 1024 + 1024;   // 8192 keys + indices
  if (shm > kMaxShm) throw Error(-1, "select: too many singular values for the on-chip sort");
  if (shm > 48 * 1024) {
    // set once per process, whichever thread gets here first
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [] {
      attr_err = hipFuncSetAttribute((const void*)select_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kMaxShm);
    });
    PTEBD_HIP(attr_err);
  }
  select_kernel<<<1, 256, shm, s>>>(vals, r, np2, is_gram, chi_max, w_max, eps, lam_out, perm, inv_sig, info_i,
                                    info_d, ledger, extra_tail);
  PTEBD_LAUNCH_CHECK();
}

void fused_row_norms(const FusedSvdArgs* tab, int count, int max_r, hipStream_t s) {
  if (count <= 0 || max_r <= 0) return;
  fused_row_norms_kernel<<<dim3(ceil_div(max_r, 4), count), 256, 0, s>>>(tab);
  PTEBD_LAUNCH_CHECK();
}

void fused_jacobi_prologue(const FusedSvdArgs* tab, int count, int max_r, double* out, hipStream_t s) {
  if (count <= 0 || max_r <= 0) return;
  fused_prologue_kernel<<<dim3(std::min(ceil_div(max_r, 256), 64), max_r + 1, count), 256, 0, s>>>(tab, out);
  PTEBD_LAUNCH_CHECK();
}

void fused_select(const FusedSvdArgs* tab, int count, int max_npow2, hipStream_t s) {
  if (count <= 0) return;
  const size_t shm = (size_t)max_npow2 * (sizeof(double) + sizeof(int));
  constexpr size_t kMaxShm = 96 * 1024 + 1024;
  if (shm > kMaxShm) throw Error(-1, "select: too many singular values for the on-chip sort");
  if (shm > 48 * 1024) {
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [] {
      attr_err = hipFuncSetAttribute((const void*)fused_select_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kMaxShm);
    });
    PTEBD_HIP(attr_err);
  }
  fused_select_kernel<<<count, 256, shm, s>>>(tab);
  PTEBD_LAUNCH_CHECK();
}

void fused_gather(const FusedSvdArgs* tab, int count, int max_k, int max_c, hipStream_t s) {
  if (count <= 0 || max_k <= 0 || max_c <= 0) return;
  fused_gather_kernel<<<dim3(std::min(ceil_div(max_c, 256), 64), max_k, count), 256, 0, s>>>(tab);
  PTEBD_LAUNCH_CHECK();
}

void gather_rows(const double* sr, const double* si, int64_t lds, const int* perm, const double* scale, int k, int c,
                 double* dr, double* di, int64_t ldd, const int* kdev, hipStream_t s) {
  (void)kdev;
  if (k <= 0 || c <= 0) return;
  dim3 g(std::min(ceil_div(c, 256), 64), k);
  gather_kernel<<<g, 256, 0, s>>>(sr, si, lds, perm, scale, k, c, dr, di, ldd);
  PTEBD_LAUNCH_CHECK();
}

}  // namespace ptebd
