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
// the off-diagonal blocks of X follow by block forward substitution.
#include "kernels.hpp"

namespace ptebd {

namespace {

constexpr int CB = 64;

// Factorises the nb x nb diagonal block at (b0, b0) of K in place (L in the
// lower triangle, zeros above) and writes its inverse into the same block of
// X.  A pivot that is not positive and finite sets *flag (the block is then
// factorised with that pivot replaced by 1, so the kernel always finishes).
__global__ __launch_bounds__(256) void chol_block_kernel(double* kr, double* ki, int64_t ld, int b0, int nb,
                                                         double* xr, double* xi, int* flag) {
  __shared__ double Ar[CB][CB + 1], Ai[CB][CB + 1];
  __shared__ double Xr[CB][CB + 1], Xi[CB][CB + 1];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < nb * nb; idx += 256) {
    const int r = idx / nb, c = idx % nb;
    const int64_t o = (int64_t)(b0 + r) * ld + b0 + c;
    Ar[r][c] = c <= r ? kr[o] : 0.0;
    Ai[r][c] = c < r ? ki[o] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (tid == 0) {
      double dj = Ar[j][j];
      if (!(dj > 0.0) || !(dj < 1e300)) {
        *flag = 1;
        dj = 1.0;
      }
      Ar[j][j] = sqrt(dj);
      Ai[j][j] = 0.0;
    }
    __syncthreads();
    const double inv = 1.0 / Ar[j][j];
    for (int i = j + 1 + tid; i < nb; i += 256) {
      Ar[i][j] *= inv;
      Ai[i][j] *= inv;
    }
    __syncthreads();
    // A(i, c) -= L(i, j) conj(L(c, j)),  j < c <= i
    const int rows = nb - j - 1;
    for (int idx = tid; idx < rows * rows; idx += 256) {
      const int i = j + 1 + idx / rows, c = j + 1 + idx % rows;
      if (c <= i) {
        const double lr = Ar[i][j], li = Ai[i][j], mr = Ar[c][j], mi = Ai[c][j];
        Ar[i][c] -= lr * mr + li * mi;
        Ai[i][c] -= li * mr - lr * mi;
      }
    }
    __syncthreads();
  }
  // X = L^-1 column by column (forward substitution; each thread one column)
  if (tid < nb) {
    const int c = tid;
    for (int i = 0; i < nb; ++i) {
      double sr = (i == c) ? 1.0 : 0.0, si = 0.0;
      if (i < c) {
        Xr[i][c] = 0.0;
        Xi[i][c] = 0.0;
        continue;
      }
      for (int p = c; p < i; ++p) {
        const double lr = Ar[i][p], li = Ai[i][p], yr = Xr[p][c], yi = Xi[p][c];
        sr -= lr * yr - li * yi;
        si -= lr * yi + li * yr;
      }
      const double d = 1.0 / Ar[i][i];
      Xr[i][c] = sr * d;
      Xi[i][c] = si * d;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < nb * nb; idx += 256) {
    const int r = idx / nb, c = idx % nb;
    const int64_t o = (int64_t)(b0 + r) * ld + b0 + c;
    kr[o] = Ar[r][c];
    ki[o] = Ai[r][c];
    xr[o] = Xr[r][c];
    xi[o] = Xi[r][c];
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
    chol_block_kernel<<<1, 256, 0, s>>>(kr, ki, ld, b0, nb, xr, xi, flag);
    PTEBD_LAUNCH_CHECK();
    const int rest = k - b0 - nb;
    if (rest <= 0) break;
    {  // panel: P = K(b0+nb:, b0:b0+nb) L_bb^-+   (rest x nb, into T with leading dimension CB)
      ZGemmArgs g;
      g.m = rest; g.n = nb; g.k = nb;
      g.ar = kr + (b0 + nb) * ld + b0; g.ai = ki + (b0 + nb) * ld + b0; g.lda = ld;
      g.br = xr + b0 * ld + b0; g.bi = xi + b0 * ld + b0; g.ldb = ld; g.transB = 1;
      g.cr = tr; g.ci = ti; g.ldc = CB;
      g.tag = "cholesky";
      zgemm(g, 0, s);
    }
    {  // trailing update: K(b0+nb:, b0+nb:) -= P P^+
      ZGemmArgs g;
      g.m = rest; g.n = rest; g.k = nb;
      g.ar = tr; g.ai = ti; g.lda = CB;
      g.br = tr; g.bi = ti; g.ldb = CB; g.transB = 1;
      g.cr = kr + (b0 + nb) * ld + b0 + nb; g.ci = ki + (b0 + nb) * ld + b0 + nb; g.ldc = ld;
      g.alpha = -1.0; g.beta = 1;
      g.tag = "cholesky";
      zgemm(g, 0, s);
    }
    // the panel of L
    scale_rows_copy(tr, ti, CB, nullptr, 1, rest, nb, kr + (b0 + nb) * ld + b0, ki + (b0 + nb) * ld + b0, ld, s);
  }
  // off-diagonal blocks of X = L^-1, row block by row block:
  // X(i, 0:i) = -X_ii L(i, 0:i) X(0:i, 0:i)
  for (int r0 = CB; r0 < k; r0 += CB) {
    const int h = std::min(CB, k - r0);
    {  // T = L(r0:r0+h, 0:r0) X(0:r0, 0:r0)   (h x r0, leading dimension k)
      ZGemmArgs g;
      g.m = h; g.n = r0; g.k = r0;
      g.ar = kr + r0 * ld; g.ai = ki + r0 * ld; g.lda = ld;
      g.br = xr; g.bi = xi; g.ldb = ld;
      g.cr = tr; g.ci = ti; g.ldc = ld;
      g.tag = "cholesky";
      zgemm(g, 0, s);
    }
    {  // X(r0:r0+h, 0:r0) = -X_ii T
      ZGemmArgs g;
      g.m = h; g.n = r0; g.k = h;
      g.ar = xr + r0 * ld + r0; g.ai = xi + r0 * ld + r0; g.lda = ld;
      g.br = tr; g.bi = ti; g.ldb = ld;
      g.cr = xr + r0 * ld; g.ci = xi + r0 * ld; g.ldc = ld;
      g.alpha = -1.0;
      g.tag = "cholesky";
      zgemm(g, 0, s);
    }
  }
}

}  // namespace ptebd
