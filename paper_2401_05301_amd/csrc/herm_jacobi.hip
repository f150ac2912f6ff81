// Two-sided block Jacobi eigensolver for a Hermitian matrix H (n x n, FP64).
//
// Used on Gram matrices, whose entries carry an absolute error of order
// u * ||H||: rotations stop once every off-diagonal entry is below
// tol_abs = c u trace(H), the accuracy the Gram matrix can support.  Blocks of
// 16 rows/columns are paired round-robin; per round:
//   herm_eig   : each pair's 32 x 32 diagonal block S = H[R, R] is
//                diagonalised in LDS by cyclic rotations, S = Q D Q^+;
//   herm_apply : every block pair (P1 >= P2) of the round is transformed,
//                H[R1, R2] <- Q1^+ H[R1, R2] Q2 (mirrored to H[R2, R1]), and
//                W[R, :] <- Q^+ W[R, :] accumulates the eigenvectors.
// At convergence H is diagonal (eigenvalues) and W H0 W^+ = H, so the rows
// of W are the conjugated eigenvectors.
#include <algorithm>
#include <cstring>

#include "kernels.hpp"
#include "profile.hpp"

namespace ptebd {

namespace {

constexpr int JB = 16;
constexpr int PR = 32;

__device__ __forceinline__ void round_pair(int nb, int t, int p, int& I, int& J) {
  auto pos = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + t) % (nb - 1); };
  int a = pos(p), b = pos(nb - 1 - p);
  I = a < b ? a : b;
  J = a < b ? b : a;
}

__device__ __forceinline__ int pidx(int I, int J, int k) { return k < JB ? I * JB + k : J * JB + (k - JB); }

__device__ __forceinline__ f64x4 mfma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// row of accumulator element e of a 16x16 FP64 MFMA result held by `lane`
__device__ __forceinline__ int acc_row(int lane, int e) { return (lane >> 4) + 4 * e; }

// Cyclic Jacobi on the 32 x 32 Hermitian block in LDS (absolute threshold).
// One step applies 16 disjoint rotations (round-robin pairs) as C <- J^+ C J
// and Q <- Q J.  For the rotation of pair k = (p, q) the 2 x 2 block of J is
//   [[cs, sn], [-sn e, cs e]],  e = conj(C_pq) / |C_pq|.
// The four entries of C at rows (p_k, q_k) and columns (p_l, q_l) depend
// only on those same four entries, so thread (k, l) of 256 updates its 2 x 2
// block of C in place, and the rows k and k + 16 of Q for pair l.  Every
// thread derives the rotations of its pairs k and l itself from the entries
// before the step (the same arithmetic on the same inputs in every thread),
// which saves a round trip through LDS and a barrier's worth of idle lanes.
struct Rot {
  double cs, sn, er, ei;
};

// cs^2 + sn^2 = 1 and |e| = 1 hold to rounding whatever the accuracy of t,
// since cs and e come from reciprocal square roots of the very quantities
// they normalise; t only sets the angle.  So t = tan(angle) is taken from
// the hardware reciprocal and reciprocal-square-root approximations, which
// shortens the dependent chain of every step: an angle off in its last bits
// leaves the rotation exactly unitary, and the remaining coupling is removed
// by the following sweeps like any other.
__device__ __forceinline__ Rot make_rot(double app, double aqq, double cre, double cim, double thr) {
  Rot r{1.0, 0.0, 1.0, 0.0};
  const double c2 = cre * cre + cim * cim;
  if (c2 > thr * thr) {
    const double rc = rsqrt(c2);   // 1 / |C_pq|
    const double tau = 0.5 * (aqq - app) * rc;
    const double at = fabs(tau);
    double t;
    if (at < 1e150) {
      // one Newton step on each hardware estimate
      const double q = 1.0 + tau * tau;
      const double y = __builtin_amdgcn_rsq(q);
      double sq = q * y;
      sq = fma(0.5 * y, fma(-sq, sq, q), sq);   // sqrt(q)
      const double den = at + sq;
      const double t0 = __builtin_amdgcn_rcp(den);
      t = fma(t0, fma(-den, t0, 1.0), t0);      // 1 / den
    } else {
      t = 0.5 / at;
    }
    t = tau >= 0.0 ? t : -t;
    r.cs = rsqrt(1.0 + t * t);
    r.sn = t * r.cs;
    r.er = cre * rc;
    r.ei = -cim * rc;
  }
  return r;
}

__device__ void block_eig(double (*Cr)[PR + 1], double (*Ci)[PR + 1], double (*Qr)[PR + 1], double (*Qi)[PR + 1],
                          double thr, int max_sweeps) {
  const int tid = threadIdx.x;
  const int k = tid >> 4, l = tid & 15;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    int changed = 0;
    for (int st = 0; st < PR - 1; ++st) {
      auto member = [st](int m) {
        if (m == 0) return 0;
        int x = m - 1 + st;
        x -= (x >= PR - 1) ? PR - 1 : 0;
        return 1 + x;
      };
      const int ka = member(k), kb = member(PR - 1 - k), la = member(l), lb = member(PR - 1 - l);
      const int p = min(ka, kb), q = max(ka, kb), u = min(la, lb), v = max(la, lb);
      const Rot rk = make_rot(Cr[p][p], Cr[q][q], Cr[p][q], Ci[p][q], thr);
      const Rot rl = make_rot(Cr[u][u], Cr[v][v], Cr[u][v], Ci[u][v], thr);
      changed |= (rk.sn != 0.0);
      __syncthreads();
      if (rk.sn != 0.0 || rl.sn != 0.0) {
        // column transform (J on the right) with pair l: col u' = cl col u - sl e_l col v,
        // col v' = sl col u + cl e_l col v; then row transform (J^+ on the left) with pair k:
        // row p' = ck row p - sk conj(e_k) row q, row q' = sk row p + ck conj(e_k) row q
        double r0r[2], r0i[2], r1r[2], r1i[2];
        const int rows[2] = {p, q};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int rr = rows[t];
          const double ur = Cr[rr][u], ui = Ci[rr][u], vr = Cr[rr][v], vi = Ci[rr][v];
          const double wr = rl.er * vr - rl.ei * vi, wi = rl.er * vi + rl.ei * vr;
          const double nur = rl.cs * ur - rl.sn * wr, nui = rl.cs * ui - rl.sn * wi;
          const double nvr = rl.sn * ur + rl.cs * wr, nvi = rl.sn * ui + rl.cs * wi;
          if (t == 0) { r0r[0] = nur; r0i[0] = nui; r0r[1] = nvr; r0i[1] = nvi; }
          else { r1r[0] = nur; r1i[0] = nui; r1r[1] = nvr; r1i[1] = nvi; }
        }
        const double ekr = rk.er, eki = -rk.ei;   // conj(e_k)
        const int cols[2] = {u, v};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const double pr_ = r0r[t], pi_ = r0i[t], qr_ = r1r[t], qi_ = r1i[t];
          const double wr = ekr * qr_ - eki * qi_, wi = ekr * qi_ + eki * qr_;
          Cr[p][cols[t]] = rk.cs * pr_ - rk.sn * wr;
          Ci[p][cols[t]] = rk.cs * pi_ - rk.sn * wi;
          Cr[q][cols[t]] = rk.sn * pr_ + rk.cs * wr;
          Ci[q][cols[t]] = rk.sn * pi_ + rk.cs * wi;
        }
      }
      if (rl.sn != 0.0) {   // Q <- Q J on rows k and k + 16, pair l
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int r = k + 16 * h;
          const double ur = Qr[r][u], ui = Qi[r][u], vr = Qr[r][v], vi = Qi[r][v];
          const double wr = rl.er * vr - rl.ei * vi, wi = rl.er * vi + rl.ei * vr;
          Qr[r][u] = rl.cs * ur - rl.sn * wr;
          Qi[r][u] = rl.cs * ui - rl.sn * wi;
          Qr[r][v] = rl.sn * ur + rl.cs * wr;
          Qi[r][v] = rl.sn * ui + rl.cs * wi;
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(changed)) break;
  }
}

// Threads per pair solve: one per (pair, pair) 2 x 2 block of the 32 x 32 block.
constexpr int kEigThreads = 256;

// Pair `pair` of the round: writes its Q (or flag 0 if the pair is already
// diagonal to the threshold).
__device__ __forceinline__ void herm_eig_pair(const HermArgs& a, int round, int pair, double (*Cr)[PR + 1],
                                              double (*Ci)[PR + 1], double (*Qr)[PR + 1], double (*Qi)[PR + 1]) {
  const int tid = threadIdx.x;
  int I, J;
  round_pair(a.nb, round, pair, I, J);
  double vc[PR * PR / kEigThreads][2];
#pragma unroll
  for (int u = 0; u < PR * PR / kEigThreads; ++u) {
    const int idx = tid + kEigThreads * u;
    const int p = idx / PR, q = idx % PR;
    const int gp = min(pidx(I, J, p), a.n - 1), gq = min(pidx(I, J, q), a.n - 1);
    vc[u][0] = a.hr[(int64_t)gp * a.ldh + gq];
    vc[u][1] = a.hi[(int64_t)gp * a.ldh + gq];
  }
#pragma unroll
  for (int u = 0; u < PR * PR / kEigThreads; ++u) {
    const int idx = tid + kEigThreads * u;
    const int p = idx / PR, q = idx % PR;
    const bool ok = pidx(I, J, p) < a.n && pidx(I, J, q) < a.n;
    Cr[p][q] = ok ? vc[u][0] : 0.0;
    Ci[p][q] = ok ? vc[u][1] : 0.0;
    Qr[p][q] = (p == q) ? 1.0 : 0.0;
    Qi[p][q] = 0.0;
  }
  __syncthreads();
  const double thr = *a.tol_abs;
  int need = 0;
  for (int idx = tid; idx < PR * PR; idx += kEigThreads) {
    const int p = idx / PR, q = idx % PR;
    if (p < q && hypot(Cr[p][q], Ci[p][q]) > thr) need = 1;
  }
  double* qout = a.qbuf + (int64_t)pair * 2 * PR * PR;
  if (!__syncthreads_or(need)) {
    if (tid == 0) a.flag[pair] = 0;
    return;
  }
  if (tid == 0) {
    a.flag[pair] = 1;
    atomicAdd(a.rotated, 1u);
  }
  block_eig(Cr, Ci, Qr, Qi, 0.5 * thr, a.inner_sweeps);
  for (int idx = tid; idx < PR * PR; idx += kEigThreads) {
    qout[idx] = Qr[idx / PR][idx % PR];
    qout[PR * PR + idx] = Qi[idx / PR][idx % PR];
  }
}

// grid: nb/2 work-groups, one pair each.
__global__ __launch_bounds__(kEigThreads) void herm_eig(HermArgs a, int round) {
  __shared__ double Cr[PR][PR + 1], Ci[PR][PR + 1], Qr[PR][PR + 1], Qi[PR][PR + 1];
  herm_eig_pair(a, round, blockIdx.x, Cr, Ci, Qr, Qi);
}

// Work-groups of one round: npairs*(npairs+1)/2 block-pair sandwiches, then
// npairs * wchunks W-row updates.
__host__ __device__ __forceinline__ int64_t apply_groups(const HermArgs& a) {
  const int64_t npairs = a.nb / 2;
  return npairs * (npairs + 1) / 2 + (a.wr ? npairs * a.wchunks : 0);
}

struct ApplyLds {
  double Ar[PR][PR + 1], Ai[PR][PR + 1], Tr[PR][PR + 1], Ti[PR][PR + 1];
  double Q1r[PR][PR + 1], Q1i[PR][PR + 1], Q2r[PR][PR + 1], Q2i[PR][PR + 1];
};

__device__ __forceinline__ void herm_apply_group(const HermArgs& a, int round, int bid, ApplyLds& L) {
  auto& Ar = L.Ar;
  auto& Ai = L.Ai;
  auto& Tr = L.Tr;
  auto& Ti = L.Ti;
  auto& Q1r = L.Q1r;
  auto& Q1i = L.Q1i;
  auto& Q2r = L.Q2r;
  auto& Q2i = L.Q2i;
  const int tid = threadIdx.x;
  const int npairs = a.nb / 2;
  const int nsand = npairs * (npairs + 1) / 2;
  if (bid < nsand) {
    // decode (P1, P2), P1 >= P2
    int P1 = 0;
    while ((P1 + 1) * (P1 + 2) / 2 <= bid) ++P1;
    const int P2 = bid - P1 * (P1 + 1) / 2;
    const int f1 = a.flag[P1], f2 = a.flag[P2];
    if (!f1 && !f2) return;
    int I1, J1, I2, J2;
    round_pair(a.nb, round, P1, I1, J1);
    round_pair(a.nb, round, P2, I2, J2);
    const double* q1 = a.qbuf + (int64_t)P1 * 2 * PR * PR;
    const double* q2 = a.qbuf + (int64_t)P2 * 2 * PR * PR;
    // Unconditional loads (indices clamped into the matrix; an unflagged
    // pair's slot holds stale but valid data), selected afterwards, so that
    // all of them are in flight together.
    double va[4][6];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = tid + 256 * u;
      const int p = idx / PR, q = idx % PR;
      const int gp = min(pidx(I1, J1, p), a.n - 1), gq = min(pidx(I2, J2, q), a.n - 1);
      va[u][0] = a.hr[(int64_t)gp * a.ldh + gq];
      va[u][1] = a.hi[(int64_t)gp * a.ldh + gq];
      va[u][2] = q1[idx];
      va[u][3] = q1[PR * PR + idx];
      va[u][4] = q2[idx];
      va[u][5] = q2[PR * PR + idx];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = tid + 256 * u;
      const int p = idx / PR, q = idx % PR;
      const bool ok = pidx(I1, J1, p) < a.n && pidx(I2, J2, q) < a.n;
      Ar[p][q] = ok ? va[u][0] : 0.0;
      Ai[p][q] = ok ? va[u][1] : 0.0;
      Q1r[p][q] = f1 ? va[u][2] : (p == q ? 1.0 : 0.0);
      Q1i[p][q] = f1 ? va[u][3] : 0.0;
      Q2r[p][q] = f2 ? va[u][4] : (p == q ? 1.0 : 0.0);
      Q2i[p][q] = f2 ? va[u][5] : 0.0;
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int tr = wave >> 1, tc = wave & 1;   // 16 x 16 output tile of this wave
    // T = Q1^+ A : A operand Q1^+(row, k) = conj(Q1(k, row)), B operand A(k, col)
    f64x4 accr = f64x4{0, 0, 0, 0}, acci = f64x4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int k = 4 * ks + (lane >> 4);
      const int row = tr * 16 + (lane & 15), col = tc * 16 + (lane & 15);
      const double xr = Q1r[k][row], xi = -Q1i[k][row];
      const double yr = Ar[k][col], yi = Ai[k][col];
      accr = mfma(xr, yr, accr);
      accr = mfma(-xi, yi, accr);
      acci = mfma(xr, yi, acci);
      acci = mfma(xi, yr, acci);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      Tr[tr * 16 + acc_row(lane, e)][tc * 16 + (lane & 15)] = accr[e];
      Ti[tr * 16 + acc_row(lane, e)][tc * 16 + (lane & 15)] = acci[e];
    }
    __syncthreads();
    // out = T Q2
    accr = f64x4{0, 0, 0, 0};
    acci = f64x4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int k = 4 * ks + (lane >> 4);
      const int row = tr * 16 + (lane & 15), col = tc * 16 + (lane & 15);
      const double xr = Tr[row][k], xi = Ti[row][k];
      const double yr = Q2r[k][col], yi = Q2i[k][col];
      accr = mfma(xr, yr, accr);
      accr = mfma(-xi, yi, accr);
      acci = mfma(xr, yi, acci);
      acci = mfma(xi, yr, acci);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int p = tr * 16 + acc_row(lane, e), q = tc * 16 + (lane & 15);
      const int gp = pidx(I1, J1, p), gq = pidx(I2, J2, q);
      double sr = accr[e], si = acci[e];
      if (gp < a.n && gq < a.n) {
        if (P1 == P2 && p == q) si = 0.0;   // keep the diagonal real
        a.hr[(int64_t)gp * a.ldh + gq] = sr;
        a.hi[(int64_t)gp * a.ldh + gq] = si;
        if (P1 != P2) {
          a.hr[(int64_t)gq * a.ldh + gp] = sr;
          a.hi[(int64_t)gq * a.ldh + gp] = -si;
        }
      }
    }
    return;
  }
  // ---- W rows update: W[R, cols] <- Q^+ W[R, cols] on the matrix cores
  bid -= nsand;
  const int P = bid / a.wchunks, ch = bid % a.wchunks;
  if (P >= npairs || !a.flag[P] || !a.wr) return;
  int I, J;
  round_pair(a.nb, round, P, I, J);
  const double* q = a.qbuf + (int64_t)P * 2 * PR * PR;
  const int lane = tid & 63, wave = tid >> 6;
  // A operand Q^+(p, k) = conj(Q(k, p)); lane: p = lane%16 (+16 t), k = 4 ks + lane/16
  double qar[2][8], qai[2][8];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int pp = t * 16 + (lane & 15), k = 4 * ks + (lane >> 4);
      qar[t][ks] = q[k * PR + pp];
      qai[t][ks] = -q[PR * PR + k * PR + pp];
    }
  const int cb = ch * a.wcols, ce = min(a.n, cb + a.wcols);
  for (int j0 = cb + wave * 16; j0 < ce; j0 += 64) {
    const int col = j0 + (lane & 15);
    const bool okc = col < ce;
    double xr[8], xi[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int row = min(pidx(I, J, 4 * ks + (lane >> 4)), a.n - 1);
      const int64_t o = (int64_t)row * a.ldw + min(col, ce - 1);
      xr[ks] = a.wr[o];
      xi[ks] = a.wi[o];
    }
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const bool ok = okc && pidx(I, J, 4 * ks + (lane >> 4)) < a.n;
      xr[ks] = ok ? xr[ks] : 0.0;
      xi[ks] = ok ? xi[ks] : 0.0;
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
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = pidx(I, J, t * 16 + acc_row(lane, e));
        if (okc && row < a.n) {
          a.wr[(int64_t)row * a.ldw + col] = orr[t][e];
          a.wi[(int64_t)row * a.ldw + col] = oii[t][e];
        }
      }
  }
}

__global__ __launch_bounds__(256) void herm_apply(HermArgs a) {
  __shared__ ApplyLds L;
  herm_apply_group(a, a.round, blockIdx.x, L);
}

// Batched form: the same round on many independent Hermitian matrices (one
// HermArgs each, in the device table tab), for the particle-number sectors
// of one SVD.  first[i] is the first work-group of matrix i (first[count] the
// total); a matrix takes part while active[i] != 0 and round < nb_i - 1 (its
// own sweep may be shorter than the longest one).
__global__ __launch_bounds__(kEigThreads) void herm_eig_batched(const HermArgs* tab, const int64_t* first, int count,
                                                                const int* active, int round) {
  __shared__ double Cr[PR][PR + 1], Ci[PR][PR + 1], Qr[PR][PR + 1], Qi[PR][PR + 1];
  const int i = batch_owner(first, count, blockIdx.x);
  const HermArgs a = tab[i];
  if (!active[i] || round >= a.nb - 1) return;
  herm_eig_pair(a, round, (int)(blockIdx.x - first[i]), Cr, Ci, Qr, Qi);
}

__global__ __launch_bounds__(256) void herm_apply_batched(const HermArgs* tab, const int64_t* first, int count,
                                                          const int* active, int round) {
  __shared__ ApplyLds L;
  const int i = batch_owner(first, count, blockIdx.x);
  const HermArgs a = tab[i];
  if (!active[i] || round >= a.nb - 1) return;
  herm_apply_group(a, round, (int)(blockIdx.x - first[i]), L);
}

// Per matrix i: number of off-diagonal entries above its threshold, into
// count[i] (grid.y = matrix).
__global__ __launch_bounds__(256) void count_above_batched_kernel(const HermArgs* tab, int count, const int* active,
                                                                  unsigned int* out) {
  const int i = blockIdx.y;
  if (i >= count || !active[i]) return;
  const HermArgs a = tab[i];
  const double t = *a.tol_abs;
  const int n = a.n;
  unsigned int c = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / n), q = (int)(e % n);
    if (r < q && hypot(a.hr[(int64_t)r * a.ldh + q], a.hi[(int64_t)r * a.ldh + q]) > t) ++c;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0 && c > 0) atomicAdd(out + i, c);
}

// Absolute off-diagonal target c u sum_i |H_ii|: for the positive
// semi-definite Gram matrices this is c units of rounding of their trace,
// the scale of the absolute error their entries carry.
__global__ __launch_bounds__(256) void trace_tol_kernel(const double* hr, int64_t ldh, int n, double c, double* out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += fabs(hr[(int64_t)i * ldh + i]);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  // floored at a tiny normal number: an exactly zero matrix needs no rotation,
  // and a target of zero would chase underflowing rounding residue
  if (threadIdx.x == 0) out[0] = fmax(c * 1.1102230246251565e-16 * sh[0], 1e-280);
}

// Largest relative coupling |H_ij| / sqrt(max(H_ii, f) max(H_jj, f)) over
// the off-diagonal entries with |H_ij| > tol, for a Hermitian positive
// semi-definite H and a floor f > 0.  Far below 1, the diagonal of H stands
// in for H itself in H^-1 (with the floor).  The value goes to *ratio_bits as
// the bit pattern of a non-negative double, so that an integer maximum
// orders it.
__global__ __launch_bounds__(256) void offdiag_ratio_kernel(const double* hr, const double* hi, int64_t ldh, int p,
                                                            const double* tol, double f,
                                                            unsigned long long* ratio_bits) {
  const double t = *tol;
  double worst = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)p * p;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / p), j = (int)(e % p);
    if (i >= j) continue;
    const double mag = hypot(hr[(int64_t)i * ldh + j], hi[(int64_t)i * ldh + j]);
    if (mag > t) {
      const double di = fmax(hr[(int64_t)i * ldh + i], f), dj = fmax(hr[(int64_t)j * ldh + j], f);
      worst = fmax(worst, mag / sqrt(di * dj));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) worst = fmax(worst, __shfl_xor(worst, off));
  if ((threadIdx.x & 63) == 0 && worst > 0.0) atomicMax(ratio_bits, (unsigned long long)__double_as_longlong(worst));
}

// Number of off-diagonal entries i < j with |H_ij| > tol (one atomic per wave).
__global__ __launch_bounds__(256) void count_above_kernel(const double* hr, const double* hi, int64_t ldh, int n,
                                                          const double* tol, unsigned int* count) {
  const double t = *tol;
  unsigned int c = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    if (i < j && hypot(hr[(int64_t)i * ldh + j], hi[(int64_t)i * ldh + j]) > t) ++c;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0 && c > 0) atomicAdd(count, c);
}

// H_ii = 0 for i < p.
__global__ void zero_diag_kernel(double* hr, double* hi, int64_t ldh, int p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p) {
    hr[(int64_t)i * ldh + i] = 0.0;
    hi[(int64_t)i * ldh + i] = 0.0;
  }
}

__global__ void set_diag_kernel(double* hr, double* hi, int64_t ldh, int p, const double* d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p) {
    hr[(int64_t)i * ldh + i] = d[i];
    hi[(int64_t)i * ldh + i] = 0.0;
  }
}

__global__ void diag_kernel(const double* hr, int64_t ldh, int n, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = hr[(int64_t)i * ldh + i];
}

}  // namespace

void herm_tol(const double* hr, int64_t ldh, int n, double c, double* out, hipStream_t s) {
  trace_tol_kernel<<<1, 256, 0, s>>>(hr, ldh, n, c, out);
  PTEBD_LAUNCH_CHECK();
}

void herm_round(HermArgs a, int round, hipStream_t s) {
  a.round = round;
  const int npairs = a.nb / 2;
  {
    ProfScope ps(K_HERM_EIG, 0.0, s);
    herm_eig<<<npairs, kEigThreads, 0, s>>>(a, round);
    PTEBD_LAUNCH_CHECK();
  }
  const int nsand = npairs * (npairs + 1) / 2;
  const int nw = a.wr ? npairs * a.wchunks : 0;
  {
    ProfScope ps(K_HERM_APPLY, 0.0, s);
    herm_apply<<<nsand + nw, 256, 0, s>>>(a);
    PTEBD_LAUNCH_CHECK();
  }
}

int64_t herm_apply_groups(const HermArgs& a) { return apply_groups(a); }

namespace {
// Every entry becomes the sum of all (one work-group, index order).
__global__ __launch_bounds__(256) void share_sum_kernel(double* v, int n) {
  __shared__ double total;
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += v[i];
    total = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256) v[i] = total;
}
}  // namespace

void share_sum(double* v, int n, hipStream_t s) {
  if (n <= 0) return;
  share_sum_kernel<<<1, 256, 0, s>>>(v, n);
  PTEBD_LAUNCH_CHECK();
}

void herm_round_batched(const HermArgs* tab, const int64_t* eig_first, int64_t eig_total, const int64_t* app_first,
                        int64_t app_total, int count, const int* active, int round, hipStream_t s) {
  {
    ProfScope ps(K_HERM_EIG, 0.0, s);
    herm_eig_batched<<<(unsigned)eig_total, kEigThreads, 0, s>>>(tab, eig_first, count, active, round);
    PTEBD_LAUNCH_CHECK();
  }
  {
    ProfScope ps(K_HERM_APPLY, 0.0, s);
    herm_apply_batched<<<(unsigned)app_total, 256, 0, s>>>(tab, app_first, count, active, round);
    PTEBD_LAUNCH_CHECK();
  }
}

void count_above_batched(const HermArgs* tab, int count, const int* active, int max_n, unsigned int* out,
                         hipStream_t s) {
  const int64_t total = (int64_t)max_n * max_n;
  dim3 g((unsigned)std::min<int64_t>((total + 255) / 256, 256), (unsigned)count);
  count_above_batched_kernel<<<g, 256, 0, s>>>(tab, count, active, out);
  PTEBD_LAUNCH_CHECK();
}

void herm_diag(const double* hr, int64_t ldh, int n, double* out, hipStream_t s) {
  diag_kernel<<<ceil_div(n, 256), 256, 0, s>>>(hr, ldh, n, out);
  PTEBD_LAUNCH_CHECK();
}

double offdiag_ratio(const double* hr, const double* hi, int64_t ldh, int p, const double* tol, double floor,
                     unsigned long long* ratio_bits, unsigned long long* h_ratio, hipStream_t s) {
  fill_zero_words(ratio_bits, 2, s);
  const int64_t n = (int64_t)p * p;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  offdiag_ratio_kernel<<<grid, 256, 0, s>>>(hr, hi, ldh, p, tol, floor, ratio_bits);
  PTEBD_LAUNCH_CHECK();
  PTEBD_HIP(hipMemcpyAsync(h_ratio, ratio_bits, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  PTEBD_HIP(hipStreamSynchronize(s));
  double v;
  std::memcpy(&v, h_ratio, sizeof(double));
  return v;
}

void set_diag(double* hr, double* hi, int64_t ldh, int p, const double* d, hipStream_t s) {
  set_diag_kernel<<<ceil_div(p, 256), 256, 0, s>>>(hr, hi, ldh, p, d);
  PTEBD_LAUNCH_CHECK();
}

void zero_diag(double* hr, double* hi, int64_t ldh, int p, hipStream_t s) {
  zero_diag_kernel<<<ceil_div(p, 256), 256, 0, s>>>(hr, hi, ldh, p);
  PTEBD_LAUNCH_CHECK();
}

unsigned int count_above(const double* hr, const double* hi, int64_t ldh, int n, const double* tol,
                         unsigned int* count, unsigned int* h_count, hipStream_t s) {
  fill_zero_words(count, 1, s);
  const int64_t total = (int64_t)n * n;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 2048);
  count_above_kernel<<<grid, 256, 0, s>>>(hr, hi, ldh, n, tol, count);
  PTEBD_LAUNCH_CHECK();
  PTEBD_HIP(hipMemcpyAsync(h_count, count, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
  PTEBD_HIP(hipStreamSynchronize(s));
  return *h_count;
}


}  // namespace ptebd
