// Element-wise, reshaping and measurement kernels (FP64).
#include "kernels.hpp"

namespace ptebd {

namespace {

__global__ void scale_rows_copy_kernel(const double* xr, const double* xi, int64_t ldx, const double* rs, int rdiv,
                                       int rows, int cols, double* yr, double* yi, int64_t ldy) {
  const int i = blockIdx.y;
  if (i >= rows) return;
  const double s = rs ? rs[i / rdiv] : 1.0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < cols; j += gridDim.x * blockDim.x) {
    yr[(int64_t)i * ldy + j] = xr[(int64_t)i * ldx + j] * s;
    yi[(int64_t)i * ldy + j] = xi[(int64_t)i * ldx + j] * s;
  }
}

// 32 x 32 tiles through LDS so that both the read and the write are coalesced.
__global__ __launch_bounds__(256) void conj_transpose_kernel(const double* xr, const double* xi, int64_t ldx,
                                                             const double* rs, int rdiv, int rows, int cols,
                                                             double* yr, double* yi, int64_t ldy) {
  __shared__ double tr[32][33], ti[32][33];
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows per pass
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + tx;
    if (i < rows && j < cols) {
      const double s = rs ? rs[i / rdiv] : 1.0;
      tr[r][tx] = xr[(int64_t)i * ldx + j] * s;
      ti[r][tx] = -xi[(int64_t)i * ldx + j] * s;
    }
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = j0 + r, i = i0 + tx;
    if (i < rows && j < cols) {
      yr[(int64_t)j * ldy + i] = tr[tx][r];
      yi[(int64_t)j * ldy + i] = ti[tx][r];
    }
  }
}

__global__ void set_identity_kernel(double* wr, double* wi, int64_t ldw, int r) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < r; j += gridDim.x * blockDim.x) {
    wr[(int64_t)i * ldw + j] = (i == j) ? 1.0 : 0.0;
    wi[(int64_t)i * ldw + j] = 0.0;
  }
}

__global__ void square_expand_kernel(const double* x, int div, int n, double* y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double v = x[i / div];
    y[i] = v * v;
  }
}

__global__ void fill_zero_kernel(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Fixed-order block reduction of one double per thread (256 threads).
__device__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// n_i = sum_{a,s,b} Lambda_i[a]^2 |B_i[a,s,b]|^2 s ; one work-group per site.
__global__ __launch_bounds__(256) void site_densities_kernel(const double* const* br, const double* const* bi,
                                                             const double* const* lam, const int* chil,
                                                             const int* chir, int d, double* n_out) {
  __shared__ double sh[4];
  const int i = blockIdx.x;
  const int cl = chil[i], cr = chir[i];
  const int64_t tot = (int64_t)cl * d * cr;
  const double* pr = br[i];
  const double* pi = bi[i];
  const double* lm = lam[i];
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < tot; e += 256) {
    const int a = (int)(e / ((int64_t)d * cr));
    const int s = (int)((e / cr) % d);
    const double l = lm[a];
    acc += l * l * (pr[e] * pr[e] + pi[e] * pi[e]) * (double)s;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) n_out[i] = t;
}

__global__ void hop_kscale_kernel(const double* lam, int cl, int d, double* ks) {
  const int rp = blockIdx.x * blockDim.x + threadIdx.x;
  const int K = cl * d - 1;
  if (rp >= K) return;
  const int r = rp + 1;
  const int a = r / d, s = r % d;
  ks[rp] = s >= 1 ? lam[a] * lam[a] * sqrt((double)s) : 0.0;
}

// sum_{y, t>=1, c} sqrt(t) conj(B(y, t-1, c)) F(y, t, c)
__global__ __launch_bounds__(256) void close_hop_kernel(const double* br, const double* bi, const double* fr,
                                                        const double* fi, int chi, int d, int cr, double* out) {
  __shared__ double sh[4];
  const int64_t tot = (int64_t)chi * (d - 1) * cr;
  double accr = 0.0, acci = 0.0;
  for (int64_t e = threadIdx.x; e < tot; e += 256) {
    const int y = (int)(e / ((int64_t)(d - 1) * cr));
    const int t = 1 + (int)((e / cr) % (d - 1));
    const int c = (int)(e % cr);
    const int64_t ob = ((int64_t)y * d + (t - 1)) * cr + c;
    const int64_t of = ((int64_t)y * d + t) * cr + c;
    const double w = sqrt((double)t);
    // conj(b) * f
    accr += w * (br[ob] * fr[of] + bi[ob] * fi[of]);
    acci += w * (br[ob] * fi[of] - bi[ob] * fr[of]);
  }
  const double sr = block_sum(accr, sh);
  const double si = block_sum(acci, sh);
  if (threadIdx.x == 0) {
    out[0] = sr;
    out[1] = si;
  }
}

}  // namespace

void scale_rows_copy(const double* xr, const double* xi, int64_t ldx, const double* rs, int rdiv, int rows, int cols,
                     double* yr, double* yi, int64_t ldy, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  dim3 g(std::min(ceil_div(cols, 256), 64), rows);
  scale_rows_copy_kernel<<<g, 256, 0, s>>>(xr, xi, ldx, rs, rdiv, rows, cols, yr, yi, ldy);
  PTEBD_LAUNCH_CHECK();
}

void conj_transpose_scaled(const double* xr, const double* xi, int64_t ldx, const double* rs, int rdiv, int rows,
                           int cols, double* yr, double* yi, int64_t ldy, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  dim3 g(ceil_div(cols, 32), ceil_div(rows, 32));
  conj_transpose_kernel<<<g, 256, 0, s>>>(xr, xi, ldx, rs, rdiv, rows, cols, yr, yi, ldy);
  PTEBD_LAUNCH_CHECK();
}

void set_identity(double* wr, double* wi, int64_t ldw, int r, hipStream_t s) {
  if (r <= 0) return;
  dim3 g(std::min(ceil_div(r, 256), 64), r);
  set_identity_kernel<<<g, 256, 0, s>>>(wr, wi, ldw, r);
  PTEBD_LAUNCH_CHECK();
}

void square_expand(const double* x, int div, int n, double* y, hipStream_t s) {
  if (n <= 0) return;
  square_expand_kernel<<<ceil_div(n, 256), 256, 0, s>>>(x, div, n, y);
  PTEBD_LAUNCH_CHECK();
}

void fill_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  fill_zero_kernel<<<std::min<int64_t>((n + 255) / 256, 4096), 256, 0, s>>>(p, n);
  PTEBD_LAUNCH_CHECK();
}

void site_densities(const double* const* br, const double* const* bi, const double* const* lam, const int* chil,
                    const int* chir, int L, int d, double* n_out, hipStream_t s) {
  site_densities_kernel<<<L, 256, 0, s>>>(br, bi, lam, chil, chir, d, n_out);
  PTEBD_LAUNCH_CHECK();
}

void hop_kscale(const double* lam, int cl, int d, double* ks, hipStream_t s) {
  const int K = cl * d - 1;
  if (K <= 0) return;
  hop_kscale_kernel<<<ceil_div(K, 256), 256, 0, s>>>(lam, cl, d, ks);
  PTEBD_LAUNCH_CHECK();
}

void close_hop(const double* br, const double* bi, const double* fr, const double* fi, int chi, int d, int cr,
               double* out, hipStream_t s) {
  close_hop_kernel<<<1, 256, 0, s>>>(br, bi, fr, fi, chi, d, cr, out);
  PTEBD_LAUNCH_CHECK();
}

}  // namespace ptebd
