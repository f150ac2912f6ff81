// Element-wise, reshaping and measurement kernels (FP64).
#include "kernels.hpp"

namespace ptebd {

namespace {

__device__ __forceinline__ void scale_rows_body(const double* xr, const double* xi, int64_t ldx, const double* rs,
                                                int rdiv, int rows, int cols, double* yr, double* yi, int64_t ldy) {
  const int i = blockIdx.y;
  if (i >= rows) return;
  const double s = rs ? rs[i / rdiv] : 1.0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < cols; j += gridDim.x * blockDim.x) {
    yr[(int64_t)i * ldy + j] = xr[(int64_t)i * ldx + j] * s;
    yi[(int64_t)i * ldy + j] = xi[(int64_t)i * ldx + j] * s;
  }
}

__global__ void scale_rows_copy_kernel(const double* xr, const double* xi, int64_t ldx, const double* rs, int rdiv,
                                       int rows, int cols, double* yr, double* yi, int64_t ldy) {
  scale_rows_body(xr, xi, ldx, rs, rdiv, rows, cols, yr, yi, ldy);
}

// 32 x 32 tiles through LDS so that both the read and the write are coalesced.
__device__ __forceinline__ void conj_transpose_body(const double* xr, const double* xi, int64_t ldx,
                                                    const double* rs, int rdiv, int rows, int cols, double* yr,
                                                    double* yi, int64_t ldy, double (*tr)[33], double (*ti)[33]) {
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

__global__ __launch_bounds__(256) void conj_transpose_kernel(const double* xr, const double* xi, int64_t ldx,
                                                             const double* rs, int rdiv, int rows, int cols,
                                                             double* yr, double* yi, int64_t ldy) {
  __shared__ double tr[32][33], ti[32][33];
  conj_transpose_body(xr, xi, ldx, rs, rdiv, rows, cols, yr, yi, ldy, tr, ti);
}

// the staging of matrix blockIdx.z of a fused batch, by its kind
__global__ void fused_scale_rows_kernel(const FusedSvdArgs* tab) {
  const FusedSvdArgs& a = tab[blockIdx.z];
  if (a.transpose) return;
  scale_rows_body(a.xr, a.xi, a.ldx, a.rs, a.rdiv, a.rows, a.cols, a.yr, a.yi, a.ldy);
}

__global__ __launch_bounds__(256) void fused_transpose_kernel(const FusedSvdArgs* tab) {
  __shared__ double tr[32][33], ti[32][33];
  const FusedSvdArgs& a = tab[blockIdx.z];
  if (!a.transpose) return;
  conj_transpose_body(a.xr, a.xi, a.ldx, a.rs, a.rdiv, a.rows, a.cols, a.yr, a.yi, a.ldy, tr, ti);
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

__global__ void fill_zero_words_kernel(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
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

// Occupation that a creation operator raises, in local state s: the site
// itself (mode 0, local dimension D = d) or the first / second physical site
// of a super site (modes 1 / 2, s = s1 d + s2).
__device__ __forceinline__ int op_level(int s, int d, int mode) { return mode == 0 ? s : (mode == 1 ? s / d : s % d); }

// ks[r'] = Lambda[a]^2 sqrt(level(s)) for the row r = r' + shift = a D + s of
// B (the row r' pairs with the state lowered by the operator), 0 when
// level(s) = 0 (the paired row then belongs to another a or level).
__global__ void op_kscale_kernel(const double* lam, int cl, int D, int d, int shift, int mode, double* ks) {
  const int rp = blockIdx.x * blockDim.x + threadIdx.x;
  const int K = cl * D - shift;
  if (rp >= K) return;
  const int r = rp + shift;
  const int a = r / D, s = r % D;
  const int lv = op_level(s, d, mode);
  ks[rp] = lv >= 1 ? lam[a] * lam[a] * sqrt((double)lv) : 0.0;
}

// sum_{y, t>=1, c} sqrt(t) conj(B(y, t-1, c)) F(y, t, c), in two passes:
// each of kHopBlocks work-groups sums a fixed slice into part[2 b], then
// one work-group adds the partial sums in block order (deterministic).
constexpr int kHopBlocks = 256;

__global__ __launch_bounds__(256) void close_hop_part_kernel(const double* br, const double* bi, const double* fr,
                                                             const double* fi, int chi, int D, int cr, int d,
                                                             int shift, int mode, double* part) {
  __shared__ double sh[4];
  const int64_t tot = (int64_t)chi * D * cr;
  double accr = 0.0, acci = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)kHopBlocks * 256) {
    const int y = (int)(e / ((int64_t)D * cr));
    const int t = (int)((e / cr) % D);
    const int c = (int)(e % cr);
    const int lv = op_level(t, d, mode);
    if (lv < 1) continue;
    const int64_t ob = ((int64_t)y * D + (t - shift)) * cr + c;
    const int64_t of = ((int64_t)y * D + t) * cr + c;
    const double w = sqrt((double)lv);
    // conj(b) * f
    accr += w * (br[ob] * fr[of] + bi[ob] * fi[of]);
    acci += w * (br[ob] * fi[of] - bi[ob] * fr[of]);
  }
  const double sr = block_sum(accr, sh);
  const double si = block_sum(acci, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr;
    part[2 * blockIdx.x + 1] = si;
  }
}

// Per super site K (one work-group each): n of its first and second
// physical site and <b+_first b_second>, from Lambda_K^2 and B_K (D = d^2):
// out[4 K ..] = (n1, n2, Re C, Im C).
__global__ __launch_bounds__(256) void supersite_local_kernel(const double* const* br, const double* const* bi,
                                                              const double* const* lam, const int* chil,
                                                              const int* chir, int d, double* out) {
  __shared__ double sh[4];
  const int K = blockIdx.x;
  const int D = d * d;
  const int cl = chil[K], cr = chir[K];
  const int64_t tot = (int64_t)cl * D * cr;
  const double* pr = br[K];
  const double* pi = bi[K];
  const double* lm = lam[K];
  double n1 = 0.0, n2 = 0.0, cre = 0.0, cim = 0.0;
  for (int64_t e = threadIdx.x; e < tot; e += 256) {
    const int a = (int)(e / ((int64_t)D * cr));
    const int t = (int)((e / cr) % D);
    const int t1 = t / d, t2 = t % d;
    const double w = lm[a] * lm[a];
    const double m2 = pr[e] * pr[e] + pi[e] * pi[e];
    n1 += w * t1 * m2;
    n2 += w * t2 * m2;
    if (t2 >= 1 && t1 + 1 < d) {
      // <s| b+_1 b_2 |t>, s = (t1 + 1, t2 - 1) = t + d - 1
      const int64_t os = e + (int64_t)(d - 1) * cr;
      const double amp = w * sqrt((double)(t1 + 1)) * sqrt((double)t2);
      cre += amp * (pr[os] * pr[e] + pi[os] * pi[e]);
      cim += amp * (pr[os] * pi[e] - pi[os] * pr[e]);
    }
  }
  const double s1 = block_sum(n1, sh);
  const double s2 = block_sum(n2, sh);
  const double s3 = block_sum(cre, sh);
  const double s4 = block_sum(cim, sh);
  if (threadIdx.x == 0) {
    out[4 * K] = s1;
    out[4 * K + 1] = s2;
    out[4 * K + 2] = s3;
    out[4 * K + 3] = s4;
  }
}

// One particle-number sector of diag(rs) A: out(i, j) = rs[r_i / rdiv] A(r_i, c_j)
// with r_i = rows[i], c_j = cols[j] (trans == 0, out m x n), or its conjugate
// transpose (trans == 1, out n x m); ldo is the leading dimension of out.
// Consecutive threads write consecutive output elements of a row.
__global__ void gather_block_kernel(const double* ar, const double* ai, int64_t lda, const double* rs, int rdiv,
                                    const int* rows, int m, const int* cols, int n, int trans, double* outr,
                                    double* outi, int64_t ldo) {
  const int64_t tot = (int64_t)m * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = trans ? (int)(e % m) : (int)(e / n);
    const int j = trans ? (int)(e / m) : (int)(e % n);
    const int r = rows[i];
    const int64_t src = (int64_t)r * lda + cols[j];
    const double sc = rs ? rs[r / rdiv] : 1.0;
    const int64_t o = trans ? (int64_t)j * ldo + i : (int64_t)i * ldo + j;
    outr[o] = ar[src] * sc;
    outi[o] = trans ? -ai[src] * sc : ai[src] * sc;
  }
}

// One work-group per entry: copies len values from (sr, si) to (dr, di),
// to dr[cols[t]] when cols is given, scaled by scale[sidx] when sidx >= 0.
__global__ __launch_bounds__(256) void rows_copy_kernel(const RowCopy* tab, const double* scale) {
  const RowCopy t = tab[blockIdx.x];
  const double sc = t.sidx >= 0 ? scale[t.sidx] : 1.0;
  for (int64_t c = threadIdx.x; c < t.len; c += 256) {
    const int64_t dst = t.cols ? (int64_t)t.cols[c] : c;
    t.dr[dst] = t.sr[c] * sc;
    t.di[dst] = t.si[c] * sc;
  }
}

__global__ void take_kernel(const double* src, const int* idx, int k, double* dst) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o < k) dst[o] = src[idx[o]];
}

__global__ __launch_bounds__(256) void close_hop_sum_kernel(const double* part, double* out) {
  __shared__ double sh[4];
  const double sr = block_sum(threadIdx.x < kHopBlocks ? part[2 * threadIdx.x] : 0.0, sh);
  const double si = block_sum(threadIdx.x < kHopBlocks ? part[2 * threadIdx.x + 1] : 0.0, sh);
  if (threadIdx.x == 0) {
    out[0] = sr;
    out[1] = si;
  }
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  // splitmix64 finaliser
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

__global__ void fill_random_kernel(double* p, int64_t n, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t h = mix64(seed ^ mix64((uint64_t)i));
    p[i] = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

__global__ __launch_bounds__(256) void normalize_rows_kernel(double* xr, double* xi, int64_t ldx, int r, int c,
                                                             double* norms) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= r) return;
  double* pr = xr + (int64_t)row * ldx;
  double* pi = xi + (int64_t)row * ldx;
  double s = 0.0;
  for (int j = lane; j < c; j += 64) s += pr[j] * pr[j] + pi[j] * pi[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  const double nrm = sqrt(s);
  if (lane == 0 && norms) norms[row] = nrm;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int j = lane; j < c; j += 64) {
    pr[j] *= inv;
    pi[j] *= inv;
  }
}

// Damped power step on Ritz pairs: row i of Y holds (G z_i)^+ and row i of Z
// holds z_i^+ with Ritz value theta_i.  The residual R_i = Y_i - theta_i Z_i
// is orthogonal to every z_j, so Y_i <- Z_i + beta_i R_i keeps the rows
// within a factor (1 + gamma^2) of orthonormal while beta_i = 1 / theta_i (a
// plain power step, up to scale) wherever the residual is small against the
// Ritz value.  Rows whose Ritz value is below zero_rel * max theta keep z_i;
// beta_i never exceeds 1 / (damp_rel * max theta).
__global__ __launch_bounds__(256) void damped_power_rows_kernel(const double* zr, const double* zi, double* yr,
                                                                double* yi, int64_t ld, int p, int r,
                                                                const double* theta, double gamma, double damp_rel,
                                                                double zero_rel) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= p) return;
  double tmax = 0.0;
  for (int j = lane; j < p; j += 64) tmax = fmax(tmax, theta[j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) tmax = fmax(tmax, __shfl_xor(tmax, off));
  const double th = theta[row];
  const double* pz = zr + (int64_t)row * ld;
  const double* qz = zi + (int64_t)row * ld;
  double* py = yr + (int64_t)row * ld;
  double* qy = yi + (int64_t)row * ld;
  double s = 0.0;
  for (int j = lane; j < r; j += 64) {
    const double a = py[j] - th * pz[j];
    const double b = qy[j] - th * qz[j];
    s += a * a + b * b;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  const double res = sqrt(s);
  double beta = 0.0;
  if (tmax > 0.0 && th > zero_rel * tmax) beta = 1.0 / fmax(fmax(th, res / gamma), damp_rel * tmax);
  const double keep = 1.0 - beta * th;
  for (int j = lane; j < r; j += 64) {
    py[j] = keep * pz[j] + beta * py[j];
    qy[j] = keep * qz[j] + beta * qy[j];
  }
}

__global__ __launch_bounds__(256) void residual_norms_kernel(const double* yr, const double* yi, const double* zr,
                                                             const double* zi, int64_t ld, int p, int r,
                                                             const double* theta, double* out) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= p) return;
  const double th = theta[row];
  const double* py = yr + (int64_t)row * ld;
  const double* qy = yi + (int64_t)row * ld;
  const double* pz = zr + (int64_t)row * ld;
  const double* qz = zi + (int64_t)row * ld;
  double s = 0.0;
  for (int j = lane; j < r; j += 64) {
    const double a = py[j] - th * pz[j];
    const double b = qy[j] - th * qz[j];
    s += a * a + b * b;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) out[row] = sqrt(s);
}

// out[e] = sum over the slices i < ns (in order) of in[i * n + e], planar.
__global__ void sum_slices_kernel(const double* ir, const double* ii, int64_t n, int ns, double* orr, double* oi) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double sr = 0.0, si = 0.0;
  for (int i = 0; i < ns; ++i) {
    sr += ir[(int64_t)i * n + e];
    si += ii[(int64_t)i * n + e];
  }
  orr[e] = sr;
  oi[e] = si;
}

// part[c * cols + j] = sum over the rows of chunk c of (rs[i / rdiv] |X_ij|)^2
__global__ __launch_bounds__(256) void col_sq_partial_kernel(const double* xr, const double* xi, int64_t ldx, int rows,
                                                             int cols, const double* rs, int rdiv, double* part) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int nch = gridDim.y, c = blockIdx.y;
  if (j >= cols) return;
  const int per = (rows + nch - 1) / nch;
  const int i0 = c * per, i1 = min(rows, i0 + per);
  double s = 0.0;
  for (int i = i0; i < i1; ++i) {
    const double w = rs ? rs[i / rdiv] : 1.0;
    const double a = xr[(int64_t)i * ldx + j] * w, b = xi[(int64_t)i * ldx + j] * w;
    s += a * a + b * b;
  }
  part[(int64_t)c * cols + j] = s;
}

// sigma_j = sqrt(sum_c part[c * cols + j]); *nrm = |sigma|; lam_j = sigma_j / |sigma|
// (one work-group, fixed summation order)
__global__ __launch_bounds__(256) void sigma_from_part_kernel(const double* part, int nch, int cols, double* lam,
                                                              double* nrm) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int j = threadIdx.x; j < cols; j += 256) {
    double t = 0.0;
    for (int c = 0; c < nch; ++c) t += part[(int64_t)c * cols + j];
    lam[j] = sqrt(t);
    acc += t;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double n = sqrt(sh[0]);
  const double inv = n > 0.0 ? 1.0 / n : 0.0;
  for (int j = threadIdx.x; j < cols; j += 256) lam[j] *= inv;
  if (threadIdx.x == 0) *nrm = n > 0.0 ? n : 1.0;
}

// X /= *nrm
__global__ void scale_recip_kernel(double* xr, double* xi, int64_t ldx, int rows, int cols, const double* nrm) {
  const double inv = 1.0 / *nrm;
  const int64_t n = (int64_t)rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols, j = e % cols;
    xr[i * ldx + j] *= inv;
    xi[i * ldx + j] *= inv;
  }
}

__global__ __launch_bounds__(256) void inv_sqrt_clamped_kernel(const double* d, int n, double rel, double* out) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) mx = fmax(mx, d[i]);
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  const double floor = rel * sh[0];
  for (int i = threadIdx.x; i < n; i += 256) out[i] = d[i] > floor ? 1.0 / sqrt(d[i]) : 0.0;
}

__global__ __launch_bounds__(256) void tail_rest_kernel(const double* hr, int64_t ldh, int n, const double* vals,
                                                        int p, double* out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += hr[(int64_t)i * ldh + i];
  for (int i = threadIdx.x; i < p; i += 256) acc -= vals[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = fmax(sh[0], 0.0);
}

// Row sums of |A_ij| of a p x p complex matrix, one wave per row.
__global__ __launch_bounds__(256) void row_abs_sums_kernel(const double* ar, const double* ai, int p, double* out) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= p) return;
  double acc = 0.0;
  for (int j = lane; j < p; j += 64) acc += hypot(ar[(int64_t)row * p + j], ai[(int64_t)row * p + j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) out[row] = acc;
}

// y = A v for a p x p complex A and complex v (planar, v at v[0..p), v[p..2p)), one wave per row.
__global__ __launch_bounds__(256) void matvec_kernel(const double* ar, const double* ai, int p, const double* v,
                                                     double* y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= p) return;
  double sr = 0.0, si = 0.0;
  for (int j = lane; j < p; j += 64) {
    const double a = ar[(int64_t)row * p + j], b = ai[(int64_t)row * p + j];
    const double x = v[j], z = v[p + j];
    sr += a * x - b * z;
    si += a * z + b * x;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off);
    si += __shfl_xor(si, off);
  }
  if (lane == 0) {
    y[row] = sr;
    y[p + row] = si;
  }
}

// v = y / |y|, *lam = |y| (one work-group).
__global__ __launch_bounds__(256) void normalize_vec_kernel(const double* y, int p, double* v, double* lam) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < 2 * p; i += 256) acc += y[i] * y[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double nrm = sqrt(sh[0]);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int i = threadIdx.x; i < 2 * p; i += 256) v[i] = y[i] * inv;
  if (threadIdx.x == 0) lam[0] = nrm;
}

// Scale for the Newton-Schulz iteration of a Hermitian positive definite A:
// c = min(Gershgorin bound, safety * power-iteration estimate), never below
// the estimate; out = (c, sqrt(c)).
__global__ __launch_bounds__(256) void ns_scale_kernel(const double* rowsums, int p, const double* lam_est,
                                                       double safety, double* out) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int i = threadIdx.x; i < p; i += 256) mx = fmax(mx, rowsums[i]);
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double c = sh[0];
    if (lam_est && safety > 0.0 && lam_est[0] > 0.0) c = fmin(c, safety * lam_est[0]);
    if (!(c > 0.0)) c = 1.0;
    out[0] = c;
    out[1] = sqrt(c);
  }
}

__global__ void ns_init_kernel(const double* ar, const double* ai, int p, const double* c, double* yr, double* yi,
                               double* zr, double* zi) {
  const double inv = 1.0 / c[0];
  const int64_t n = (int64_t)p * p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    yr[e] = ar[e] * inv;
    yi[e] = ai[e] * inv;
    zr[e] = (e / p == e % p) ? 1.0 : 0.0;
    zi[e] = 0.0;
  }
}

__global__ __launch_bounds__(256) void ns_three_minus_kernel(double* pr, double* pi, int p, double* dev) {
  __shared__ double sh[256];
  const int64_t n = (int64_t)p * p;
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const bool dg = (e / p == e % p);
    const double tr = (dg ? 1.5 : 0.0) - 0.5 * pr[e];
    const double ti = -0.5 * pi[e];
    const double dr = tr - (dg ? 1.0 : 0.0);
    acc += dr * dr + ti * ti;
    pr[e] = tr;
    pi[e] = ti;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dev[blockIdx.x] = sh[0];   // per-block partial, summed in order by the host
}

}  // namespace

// Adds the per-gate ledger slots to the running total in gate order, so that
// the sum does not depend on which worker finished first.
__global__ void accumulate_slots_kernel(const double* slots, int n, double* acc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t = 0.0;
  for (int i = 0; i < n; ++i) t += slots[i];
  acc[0] += t;
}

void ns_scale(const double* ar, const double* ai, int p, double* work, int power_its, double safety, double* out,
              hipStream_t s) {
  // work: row sums [p], v [2p], y [2p], lambda [1]
  double* rows = work;
  double* v = work + p;
  double* y = work + 3 * p;
  double* lam = work + 5 * p;
  hipLaunchKernelGGL(row_abs_sums_kernel, dim3(ceil_div(p, 4)), dim3(256), 0, s, ar, ai, p, rows);
  PTEBD_LAUNCH_CHECK();
  if (power_its > 0) {
    fill_random(v, 2 * (int64_t)p, 0x9e3779b97f4a7c15ull, s);
    for (int it = 0; it < power_its; ++it) {
      hipLaunchKernelGGL(matvec_kernel, dim3(ceil_div(p, 4)), dim3(256), 0, s, ar, ai, p, v, y);
      PTEBD_LAUNCH_CHECK();
      hipLaunchKernelGGL(normalize_vec_kernel, dim3(1), dim3(256), 0, s, y, p, v, lam);
      PTEBD_LAUNCH_CHECK();
    }
  }
  hipLaunchKernelGGL(ns_scale_kernel, dim3(1), dim3(256), 0, s, rows, p, power_its > 0 ? lam : nullptr, safety, out);
  PTEBD_LAUNCH_CHECK();
}

void ns_init(const double* ar, const double* ai, int p, const double* c, double* yr, double* yi, double* zr,
             double* zi, hipStream_t s) {
  ns_init_kernel<<<std::min<int64_t>(((int64_t)p * p + 255) / 256, 2048), 256, 0, s>>>(ar, ai, p, c, yr, yi, zr, zi);
  PTEBD_LAUNCH_CHECK();
}

int ns_three_minus(double* pr, double* pi, int p, double* dev, hipStream_t s) {
  const int g = (int)std::min<int64_t>(((int64_t)p * p + 255) / 256, 256);
  ns_three_minus_kernel<<<g, 256, 0, s>>>(pr, pi, p, dev);
  PTEBD_LAUNCH_CHECK();
  return g;
}

void fill_random(double* p, int64_t n, uint64_t seed, hipStream_t s) {
  if (n <= 0) return;
  fill_random_kernel<<<std::min<int64_t>((n + 255) / 256, 4096), 256, 0, s>>>(p, n, seed);
  PTEBD_LAUNCH_CHECK();
}

void normalize_rows(double* xr, double* xi, int64_t ldx, int r, int c, double* norms, hipStream_t s) {
  if (r <= 0) return;
  normalize_rows_kernel<<<ceil_div(r, 4), 256, 0, s>>>(xr, xi, ldx, r, c, norms);
  PTEBD_LAUNCH_CHECK();
}

void inv_sqrt_clamped(const double* d, int n, double rel, double* out, hipStream_t s) {
  inv_sqrt_clamped_kernel<<<1, 256, 0, s>>>(d, n, rel, out);
  PTEBD_LAUNCH_CHECK();
}

void tail_rest(const double* hr, int64_t ldh, int n, const double* vals, int p, double* out, hipStream_t s) {
  tail_rest_kernel<<<1, 256, 0, s>>>(hr, ldh, n, vals, p, out);
  PTEBD_LAUNCH_CHECK();
}

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

void fused_stage(const FusedSvdArgs* tab, int count, int max_rows, int max_cols, hipStream_t s) {
  if (count <= 0 || max_rows <= 0 || max_cols <= 0) return;
  fused_scale_rows_kernel<<<dim3(std::min(ceil_div(max_cols, 256), 64), max_rows, count), 256, 0, s>>>(tab);
  PTEBD_LAUNCH_CHECK();
  fused_transpose_kernel<<<dim3(ceil_div(max_cols, 32), ceil_div(max_rows, 32), count), 256, 0, s>>>(tab);
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

void fill_zero_words(void* p, int64_t words, hipStream_t s) {
  if (words <= 0) return;
  fill_zero_words_kernel<<<std::min<int64_t>((words + 255) / 256, 4096), 256, 0, s>>>(static_cast<uint32_t*>(p),
                                                                                   words);
  PTEBD_LAUNCH_CHECK();
}

void site_densities(const double* const* br, const double* const* bi, const double* const* lam, const int* chil,
                    const int* chir, int L, int d, double* n_out, hipStream_t s) {
  site_densities_kernel<<<L, 256, 0, s>>>(br, bi, lam, chil, chir, d, n_out);
  PTEBD_LAUNCH_CHECK();
}

void op_kscale(const double* lam, int cl, int D, int d, int shift, int mode, double* ks, hipStream_t s) {
  const int K = cl * D - shift;
  if (K <= 0) return;
  op_kscale_kernel<<<ceil_div(K, 256), 256, 0, s>>>(lam, cl, D, d, shift, mode, ks);
  PTEBD_LAUNCH_CHECK();
}

void close_op(const double* br, const double* bi, const double* fr, const double* fi, int chi, int D, int cr, int d,
              int shift, int mode, double* out, double* part, hipStream_t s) {
  close_hop_part_kernel<<<kHopBlocks, 256, 0, s>>>(br, bi, fr, fi, chi, D, cr, d, shift, mode, part);
  PTEBD_LAUNCH_CHECK();
  close_hop_sum_kernel<<<1, 256, 0, s>>>(part, out);
  PTEBD_LAUNCH_CHECK();
}

void gather_block(const double* ar, const double* ai, int64_t lda, const double* rs, int rdiv, const int* rows, int m,
                  const int* cols, int n, int trans, double* outr, double* outi, int64_t ldo, hipStream_t s) {
  const int64_t tot = (int64_t)m * n;
  if (tot <= 0) return;
  gather_block_kernel<<<(int)std::min<int64_t>((tot + 255) / 256, 8192), 256, 0, s>>>(
      ar, ai, lda, rs, rdiv, rows, m, cols, n, trans, outr, outi, ldo);
  PTEBD_LAUNCH_CHECK();
}

void rows_copy(const RowCopy* tab, int count, const double* scale, hipStream_t s) {
  if (count <= 0) return;
  rows_copy_kernel<<<count, 256, 0, s>>>(tab, scale);
  PTEBD_LAUNCH_CHECK();
}

void take(const double* src, const int* idx, int k, double* dst, hipStream_t s) {
  if (k <= 0) return;
  take_kernel<<<ceil_div(k, 256), 256, 0, s>>>(src, idx, k, dst);
  PTEBD_LAUNCH_CHECK();
}

void supersite_local(const double* const* br, const double* const* bi, const double* const* lam, const int* chil,
                     const int* chir, int Ls, int d, double* out, hipStream_t s) {
  supersite_local_kernel<<<Ls, 256, 0, s>>>(br, bi, lam, chil, chir, d, out);
  PTEBD_LAUNCH_CHECK();
}

void accumulate_slots(const double* slots, int n, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(accumulate_slots_kernel, dim3(1), dim3(64), 0, s, slots, n, acc);
  PTEBD_LAUNCH_CHECK();
}

void refine_sigma(double* xr, double* xi, int64_t ldx, int rows, int cols, const double* rs, int rdiv, double* part,
                  int64_t part_cap, double* lam, double* nrm, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  int nch = std::min(64, rows);
  while (nch > 1 && (int64_t)nch * cols > part_cap) nch /= 2;
  if ((int64_t)nch * cols > part_cap) throw Error(-1, "refine_sigma: scratch too small");
  col_sq_partial_kernel<<<dim3(ceil_div(cols, 256), nch), 256, 0, s>>>(xr, xi, ldx, rows, cols, rs, rdiv, part);
  PTEBD_LAUNCH_CHECK();
  sigma_from_part_kernel<<<1, 256, 0, s>>>(part, nch, cols, lam, nrm);
  PTEBD_LAUNCH_CHECK();
  const int64_t n = (int64_t)rows * cols;
  scale_recip_kernel<<<(unsigned)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, s>>>(xr, xi, ldx, rows, cols,
                                                                                      nrm);
  PTEBD_LAUNCH_CHECK();
}

void residual_norms(const double* yr, const double* yi, const double* zr, const double* zi, int64_t ld, int p, int r,
                    const double* theta, double* out, hipStream_t s) {
  residual_norms_kernel<<<ceil_div(p, 4), 256, 0, s>>>(yr, yi, zr, zi, ld, p, r, theta, out);
  PTEBD_LAUNCH_CHECK();
}

void sum_slices(const double* ir, const double* ii, int64_t n, int ns, double* orr, double* oi, hipStream_t s) {
  if (n <= 0) return;
  sum_slices_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ir, ii, n, ns, orr, oi);
  PTEBD_LAUNCH_CHECK();
}

void damped_power_rows(const double* zr, const double* zi, double* yr, double* yi, int64_t ld, int p, int r,
                       const double* theta, double gamma, double damp_rel, double zero_rel, hipStream_t s) {
  hipLaunchKernelGGL(damped_power_rows_kernel, dim3(ceil_div(p, 4)), dim3(256), 0, s, zr, zi, yr, yi, ld, p, r, theta,
                     gamma, damp_rel, zero_rel);
  PTEBD_LAUNCH_CHECK();
}

}  // namespace ptebd
