// Blocked Cholesky factorisation and triangular inverse of a Hermitian
// positive definite matrix (planar FP64), for Cholesky-QR orthonormalisation
// of the rows of a matrix whose Gram matrix is close to the identity.
//
// K (k x k, lower triangle used) = L L^+ with L lower triangular; X = L^-1.
// The rows of L^-1 V are orthonormal when K = V V^+, and row i of L^-1 V is a
// combination of rows 0..i of V only (Gram-Schmidt in row order).
//
// Blocks of 64: each diagonal block is factorised and inverted in LDS by one
// work-group; the panel below it and the trailing update are complex GEMMs;
// the off-diagonal blocks of X follow by recursive doubling over the blocks.
#include <utility>
#include <vector>

#include "kernels.hpp"

namespace ptebd {

namespace {

constexpr int CB = 64;
constexpr int kBlockThreads = 1024;   // 64 rows x 16 column lanes

// Factorises the nb x nb diagonal block at (b0, b0) of K in place (L in the
// lower triangle, zeros above) and writes its inverse into the same block of
// X.  A pivot that is not positive and finite sets *flag (the block is then
// factorised with that pivot replaced by 1, so the kernel always finishes).
//
// Right-looking factorisation on unscaled columns: step j subtracts
// a_ij conj(a_cj) / a_jj from every trailing entry (c <= i), which reads
// only column j and the pivot, so one barrier per column suffices; the
// columns are scaled by 1 / sqrt(a_jj) afterwards.  The inverse follows by
// the same right-looking pattern: row p of X is final once the earlier rows
// have been subtracted, and is scaled at the end.  Thread (r, q) of 64 x 16
// owns row r and every sixteenth column of the trailing block.
__device__ __forceinline__ double fixed_pivot(double d) { return (d > 0.0 && d < 1e300) ? d : 1.0; }

__global__ __launch_bounds__(kBlockThreads) void chol_block_kernel(double* kr, double* ki, int64_t ld, int b0, int nb,
                                                                   double* xr, double* xi, int* flag) {
  __shared__ double Ar[CB][CB + 1], Ai[CB][CB + 1];
  __shared__ double Xr[CB][CB + 1], Xi[CB][CB + 1];
  const int tid = threadIdx.x;
  const int r = tid >> 4, q = tid & 15;
  for (int idx = tid; idx < nb * nb; idx += kBlockThreads) {
    const int i = idx / nb, c = idx % nb;
    const int64_t o = (int64_t)(b0 + i) * ld + b0 + c;
    Ar[i][c] = c <= i ? kr[o] : 0.0;
    Ai[i][c] = c < i ? ki[o] : 0.0;
    Xr[i][c] = i == c ? 1.0 : 0.0;
    Xi[i][c] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j + 1 < nb; ++j) {
    const double rd = 1.0 / fixed_pivot(Ar[j][j]);
    const int i = j + 1 + r;
    if (i < nb) {
      const double lr = Ar[i][j] * rd, li = Ai[i][j] * rd;
      for (int c = j + 1 + q; c <= i; c += 16) {
        const double mr = Ar[c][j], mi = Ai[c][j];
        Ar[i][c] -= lr * mr + li * mi;
        Ai[i][c] -= li * mr - lr * mi;
      }
    }
    __syncthreads();
  }
  if (tid == 0)
    for (int j = 0; j < nb; ++j)
      if (!(Ar[j][j] > 0.0 && Ar[j][j] < 1e300)) *flag = 1;
  // scale column c by 1 / sqrt(pivot) (rows below the diagonal), pivot -> sqrt
  for (int idx = tid; idx < nb * nb; idx += kBlockThreads) {
    const int i = idx / nb, c = idx % nb;
    if (i > c) {
      const double s = 1.0 / sqrt(fixed_pivot(Ar[c][c]));
      Ar[i][c] *= s;
      Ai[i][c] *= s;
    }
  }
  __syncthreads();
  if (tid < nb) {
    Ar[tid][tid] = sqrt(fixed_pivot(Ar[tid][tid]));
    Ai[tid][tid] = 0.0;
  }
  __syncthreads();
  // X = L^-1: step p subtracts l_ip x_pc / l_pp from rows i > p (columns c <= p)
  for (int p = 0; p + 1 < nb; ++p) {
    const int i = p + 1 + r;
    if (i < nb) {
      const double d = 1.0 / Ar[p][p];
      const double lr = Ar[i][p] * d, li = Ai[i][p] * d;
      for (int c = q; c <= p; c += 16) {
        const double yr = Xr[p][c], yi = Xi[p][c];
        Xr[i][c] -= lr * yr - li * yi;
        Xi[i][c] -= lr * yi + li * yr;
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nb * nb; idx += kBlockThreads) {
    const int i = idx / nb, c = idx % nb;
    const int64_t o = (int64_t)(b0 + i) * ld + b0 + c;
    const double d = 1.0 / Ar[i][i];
    kr[o] = Ar[i][c];
    ki[o] = Ai[i][c];
    xr[o] = Xr[i][c] * d;
    xi[o] = Xi[i][c] * d;
  }
}

}  // namespace

void chol_inverse(double* kr, double* ki, int k, double* xr, double* xi, double* tr, double* ti, int* flag,
                  hipStream_t s) {
  if (k <= 0) return;
  const int64_t ld = k;
  fill_zero(xr, (int64_t)k * k, s);
  fill_zero(xi, (int64_t)k * k, s);
  for (int b0 = 0; b0 < k; b0 += CB) {
    const int nb = std::min(CB, k - b0);
    chol_block_kernel<<<1, kBlockThreads, 0, s>>>(kr, ki, ld, b0, nb, xr, xi, flag);
    PTEBD_LAUNCH_CHECK();
    const int rest = k - b0 - nb;
    if (rest <= 0) break;
    {  // panel in place: L(b0+nb:, b0:b0+nb) = K(b0+nb:, b0:b0+nb) L_bb^-+.  Each
       // 64-row output tile is read only by the work-group that writes it, and
       // written after its last read, so the product may overwrite its operand.
      ZGemmArgs g;
      g.m = rest; g.n = nb; g.k = nb;
      g.ar = kr + (b0 + nb) * ld + b0; g.ai = ki + (b0 + nb) * ld + b0; g.lda = ld;
      g.br = xr + b0 * ld + b0; g.bi = xi + b0 * ld + b0; g.ldb = ld; g.transB = 1;
      g.cr = kr + (b0 + nb) * ld + b0; g.ci = ki + (b0 + nb) * ld + b0; g.ldc = ld;
      g.tag = "cholesky";
      zgemm(g, 0, s);
    }
    {  // trailing update: K(b0+nb:, b0+nb:) -= L_panel L_panel^+
      ZGemmArgs g;
      g.m = rest; g.n = rest; g.k = nb;
      g.ar = kr + (b0 + nb) * ld + b0; g.ai = ki + (b0 + nb) * ld + b0; g.lda = ld;
      g.br = kr + (b0 + nb) * ld + b0; g.bi = ki + (b0 + nb) * ld + b0; g.ldb = ld; g.transB = 1;
      g.cr = kr + (b0 + nb) * ld + b0 + nb; g.ci = ki + (b0 + nb) * ld + b0 + nb; g.ldc = ld;
      g.alpha = -1.0; g.beta = 1;
      g.tag = "cholesky";
      zgemm(g, 0, s);
    }
  }
  // Off-diagonal blocks of X = L^-1 by recursive doubling: two neighbouring
  // segments A (before) and B whose diagonal blocks of X are complete give
  //   X(B, A) = -X(B, B) L(B, A) X(A, A),
  // which completes the segment A u B.  The merges of one level are
  // independent; those of equal-sized segments run as one batched product
  // (T, at the same place in the scratch, holds L(B, A) X(A, A)).
  std::vector<std::pair<int, int>> seg;   // (start, length)
  for (int b0 = 0; b0 < k; b0 += CB) seg.push_back({b0, std::min(CB, k - b0)});
  auto merge = [&](int a0, int n1, int n2, int batch, int64_t stride) {
    const int b0 = a0 + n1;
    ZGemmArgs g;   // T = L(B, A) X(A, A)
    g.m = n2; g.n = n1; g.k = n1; g.batch = batch;
    g.ar = kr + b0 * ld + a0; g.ai = ki + b0 * ld + a0; g.lda = ld; g.sA = stride;
    g.br = xr + a0 * ld + a0; g.bi = xi + a0 * ld + a0; g.ldb = ld; g.sB = stride;
    g.cr = tr + b0 * ld + a0; g.ci = ti + b0 * ld + a0; g.ldc = ld; g.sC = stride;
    g.tag = "cholesky";
    zgemm(g, 0, s);
    ZGemmArgs h;   // X(B, A) = -X(B, B) T
    h.m = n2; h.n = n1; h.k = n2; h.batch = batch;
    h.ar = xr + b0 * ld + b0; h.ai = xi + b0 * ld + b0; h.lda = ld; h.sA = stride;
    h.br = tr + b0 * ld + a0; h.bi = ti + b0 * ld + a0; h.ldb = ld; h.sB = stride;
    h.cr = xr + b0 * ld + a0; h.ci = xi + b0 * ld + a0; h.ldc = ld; h.sC = stride;
    h.alpha = -1.0;
    h.tag = "cholesky";
    zgemm(h, 0, s);
  };
  while (seg.size() > 1) {
    std::vector<std::pair<int, int>> next;
    const size_t pairs = seg.size() / 2;
    // leading run of pairs whose two segments both have the first segment's length
    const int len = seg[0].second;
    size_t uniform = 0;
    while (uniform < pairs && seg[2 * uniform].second == len && seg[2 * uniform + 1].second == len) ++uniform;
    if (uniform > 0) merge(seg[0].first, len, len, (int)uniform, 2 * (int64_t)len * (ld + 1));
    for (size_t m = uniform; m < pairs; ++m) merge(seg[2 * m].first, seg[2 * m].second, seg[2 * m + 1].second, 1, 0);
    for (size_t m = 0; m < pairs; ++m) next.push_back({seg[2 * m].first, seg[2 * m].second + seg[2 * m + 1].second});
    if (seg.size() & 1) next.push_back(seg.back());
    seg.swap(next);
  }
}

}  // namespace ptebd
