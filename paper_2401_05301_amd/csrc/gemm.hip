// Complex planar GEMM on the gfx950 matrix cores.
//
// One work-group of 256 threads (four wave64) computes a 64 x 64 tile of C;
// each wave owns a 32 x 32 quadrant as 2 x 2 MFMA tiles of 16 x 16.  The
// complex product is four real products (Cr += Ar Br - Ai Bi,
// Ci += Ar Bi + Ai Br), so both rounding errors stay symmetric.  K is walked
// in slabs of 16 staged through LDS.  Precisions:
//   FP64  : v_mfma_f64_16x16x4_f64
//   FP32  : operands rounded to FP32, v_mfma_f32_16x16x4_f32, FP32 accumulation
//   SPLIT : x = hi + lo with hi = fl32(x), lo = fl32(x - hi); products
//           hi*hi + hi*lo + lo*hi, FP32 accumulation.
#include <type_traits>

#include "kernels.hpp"
#include "profile.hpp"

namespace ptebd {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, PAD = 1;

__device__ __forceinline__ f64x4 mfma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int PREC>
struct Traits {
  using T = std::conditional_t<PREC == 0, double, float>;
  using Acc = std::conditional_t<PREC == 0, f64x4, f32x4>;
  static constexpr int NPART = PREC == 2 ? 2 : 1;  // hi (and lo) planes
};

template <int PREC>
__device__ __forceinline__ void put(typename Traits<PREC>::T (*s)[BK][BM + PAD], int kk, int r, double v) {
  if constexpr (PREC == 0) {
    s[0][kk][r] = v;
  } else if constexpr (PREC == 1) {
    s[0][kk][r] = (float)v;
  } else {
    float hi = (float)v;
    s[0][kk][r] = hi;
    s[1][kk][r] = (float)(v - (double)hi);
  }
}

template <int PREC>
__global__ __launch_bounds__(256) void zgemm_kernel(ZGemmArgs g) {
  using Tr = Traits<PREC>;
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  constexpr int NP = Tr::NPART;
  __shared__ T As_r[NP][BK][BM + PAD], As_i[NP][BK][BM + PAD];
  __shared__ T Bs_r[NP][BK][BN + PAD], Bs_i[NP][BK][BN + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t bz = blockIdx.z;
  int tile_r = blockIdx.y, tile_c = blockIdx.x;
  if (g.herm_out) {
    // lower-triangular tiles only (tile_c <= tile_r), linearised in blockIdx.x
    const int t = blockIdx.x;
    int ty = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((ty + 1) * (ty + 2) / 2 <= t) ++ty;
    while (ty * (ty + 1) / 2 > t) --ty;
    tile_r = ty;
    tile_c = t - ty * (ty + 1) / 2;
  }
  const int row0 = tile_r * BM, col0 = tile_c * BN;
  const double* Ar = g.ar + bz * g.sA;
  const double* Ai = g.ai + bz * g.sA;
  const double* Br = g.br + bz * g.sB;
  const double* Bi = g.bi + bz * g.sB;

  Acc accr[2][2], acci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accr[a][b] = Acc{0, 0, 0, 0};
      acci[a][b] = Acc{0, 0, 0, 0};
    }

  // Global loads of the next K slab go to registers while the current slab is
  // multiplied out of LDS (register double buffering).
  double ra_r[4], ra_i[4], rb_r[4], rb_i[4];
  auto load = [&](int k0) {
    if (!g.transA) {
      const int kk = tid & 15, kg = k0 + kk;
      const double ks = (g.k_scale && kg < g.k) ? g.k_scale[kg / g.k_div] : 1.0;
#pragma unroll
      for (int rep = 0; rep < 4; ++rep) {
        const int i = row0 + (tid >> 4) + 16 * rep;
        const bool ok = i < g.m && kg < g.k;
        const int64_t o = (int64_t)i * g.lda + kg;
        ra_r[rep] = ok ? Ar[o] * ks : 0.0;
        ra_i[rep] = ok ? Ai[o] * ks : 0.0;
      }
    } else {
      const int i = row0 + (tid & 63);
#pragma unroll
      for (int rep = 0; rep < 4; ++rep) {
        const int kg = k0 + (tid >> 6) + 4 * rep;
        const bool ok = i < g.m && kg < g.k;
        const double ks = (ok && g.k_scale) ? g.k_scale[kg / g.k_div] : 1.0;
        const int64_t o = (int64_t)kg * g.lda + i;
        ra_r[rep] = ok ? Ar[o] * ks : 0.0;
        ra_i[rep] = ok ? -Ai[o] * ks : 0.0;
      }
    }
    if (!g.transB) {
      const int j = col0 + (tid & 63);
#pragma unroll
      for (int rep = 0; rep < 4; ++rep) {
        const int kg = k0 + (tid >> 6) + 4 * rep;
        const bool ok = j < g.n && kg < g.k;
        const int64_t o = (int64_t)kg * g.ldb + j;
        rb_r[rep] = ok ? Br[o] : 0.0;
        rb_i[rep] = ok ? Bi[o] : 0.0;
      }
    } else {
      const int kg = k0 + (tid & 15);
#pragma unroll
      for (int rep = 0; rep < 4; ++rep) {
        const int j = col0 + (tid >> 4) + 16 * rep;
        const bool ok = j < g.n && kg < g.k;
        const int64_t o = (int64_t)j * g.ldb + kg;
        rb_r[rep] = ok ? Br[o] : 0.0;
        rb_i[rep] = ok ? -Bi[o] : 0.0;
      }
    }
  };
  auto stage = [&]() {
    if (!g.transA) {
#pragma unroll
      for (int rep = 0; rep < 4; ++rep) {
        put<PREC>(As_r, tid & 15, (tid >> 4) + 16 * rep, ra_r[rep]);
        put<PREC>(As_i, tid & 15, (tid >> 4) + 16 * rep, ra_i[rep]);
      }
    } else {
#pragma unroll
      for (int rep = 0; rep < 4; ++rep) {
        put<PREC>(As_r, (tid >> 6) + 4 * rep, tid & 63, ra_r[rep]);
        put<PREC>(As_i, (tid >> 6) + 4 * rep, tid & 63, ra_i[rep]);
      }
    }
    if (!g.transB) {
#pragma unroll
      for (int rep = 0; rep < 4; ++rep) {
        put<PREC>(Bs_r, (tid >> 6) + 4 * rep, tid & 63, rb_r[rep]);
        put<PREC>(Bs_i, (tid >> 6) + 4 * rep, tid & 63, rb_i[rep]);
      }
    } else {
#pragma unroll
      for (int rep = 0; rep < 4; ++rep) {
        put<PREC>(Bs_r, tid & 15, (tid >> 4) + 16 * rep, rb_r[rep]);
        put<PREC>(Bs_i, tid & 15, (tid >> 4) + 16 * rep, rb_i[rep]);
      }
    }
  };

  load(0);
  for (int k0 = 0; k0 < g.k; k0 += BK) {
    stage();
    __syncthreads();
    if (k0 + BK < g.k) load(k0 + BK);

#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T ar[NP][2], ai[NP][2], br[NP][2], bi[NP][2];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          ar[p][t] = As_r[p][kr][wm * 32 + t * 16 + (lane & 15)];
          ai[p][t] = As_i[p][kr][wm * 32 + t * 16 + (lane & 15)];
          br[p][t] = Bs_r[p][kr][wn * 32 + t * 16 + (lane & 15)];
          bi[p][t] = Bs_i[p][kr][wn * 32 + t * 16 + (lane & 15)];
        }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if constexpr (PREC != 2) {
            accr[a][b] = mfma(ar[0][a], br[0][b], accr[a][b]);
            accr[a][b] = mfma(-ai[0][a], bi[0][b], accr[a][b]);
            acci[a][b] = mfma(ar[0][a], bi[0][b], acci[a][b]);
            acci[a][b] = mfma(ai[0][a], br[0][b], acci[a][b]);
          } else {
            // hi*hi + hi*lo + lo*hi for each of the four real products
            accr[a][b] = mfma(ar[0][a], br[0][b], accr[a][b]);
            accr[a][b] = mfma(ar[0][a], br[1][b], accr[a][b]);
            accr[a][b] = mfma(ar[1][a], br[0][b], accr[a][b]);
            accr[a][b] = mfma(-ai[0][a], bi[0][b], accr[a][b]);
            accr[a][b] = mfma(-ai[0][a], bi[1][b], accr[a][b]);
            accr[a][b] = mfma(-ai[1][a], bi[0][b], accr[a][b]);
            acci[a][b] = mfma(ar[0][a], bi[0][b], acci[a][b]);
            acci[a][b] = mfma(ar[0][a], bi[1][b], acci[a][b]);
            acci[a][b] = mfma(ar[1][a], bi[0][b], acci[a][b]);
            acci[a][b] = mfma(ai[0][a], br[0][b], acci[a][b]);
            acci[a][b] = mfma(ai[0][a], br[1][b], acci[a][b]);
            acci[a][b] = mfma(ai[1][a], br[0][b], acci[a][b]);
          }
        }
    }
    __syncthreads();
  }

  // ---- epilogue: scalings, store.  16x16 MFMA output: lane holds column lane%16;
  // element e sits in row 4*(lane/16) + e for the FP32 product and in row
  // lane/16 + 4*e for the FP64 product.
  double alpha = g.alpha;
  if (g.alpha_dev) alpha *= g.alpha_recip ? 1.0 / g.alpha_dev[0] : g.alpha_dev[0];
  double* Cr = g.cr + bz * g.sC;
  double* Ci = g.ci + bz * g.sC;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = row0 + wm * 32 + a * 16 + (PREC == 0 ? (lane >> 4) + 4 * e : 4 * (lane >> 4) + e);
        const int j = col0 + wn * 32 + b * 16 + (lane & 15);
        if (i < g.m && j < g.n) {
          double s = alpha;
          if (g.row_scale) s *= g.row_scale[i / g.row_div];
          if (g.col_scale) s *= g.col_scale[j / g.col_div];
          const double vr = (double)accr[a][b][e] * s, vi = (double)acci[a][b][e] * s;
          const int64_t o = (int64_t)i * g.ldc + j;
          if (g.beta) {
            Cr[o] += vr;
            Ci[o] += vi;
          } else {
            Cr[o] = vr;
            Ci[o] = vi;
          }
          if (g.herm_out && tile_c < tile_r) {   // mirror into the upper triangle
            const int64_t om = (int64_t)j * g.ldc + i;
            Cr[om] = vr;
            Ci[om] = -vi;
          }
        }
      }
}

}  // namespace

void zgemm(const ZGemmArgs& a, int prec, hipStream_t s) {
  if (a.m <= 0 || a.n <= 0 || a.batch <= 0) return;
  if (a.k <= 0) throw Error(-1, "zgemm: k must be positive");
  dim3 grid(ceil_div(a.n, BN), ceil_div(a.m, BM), a.batch);
  if (a.herm_out) {
    // C = X X^+ is Hermitian: only tiles on or below the diagonal are computed
    if (a.m != a.n || a.beta || a.col_scale != a.row_scale || a.col_div != a.row_div)
      throw Error(-1, "zgemm: Hermitian output needs a square, overwritten, symmetrically scaled C");
    const int T = ceil_div(a.m, BM);
    grid = dim3(T * (T + 1) / 2, 1, a.batch);
  }
  if (grid.y > 65535 || grid.z > 65535) throw Error(-1, "zgemm: grid too large");
  // algorithmic work: a Hermitian Gram product counts as a rank-k update
  const double flops = a.herm_out ? 4.0 * a.m * a.m * (double)a.k * a.batch
                                  : 8.0 * a.m * (double)a.n * a.k * a.batch;
  ProfScope ps(prec == 0 ? K_GEMM_FP64 : K_GEMM_FP32, flops, s);
  switch (prec) {
    case 0: zgemm_kernel<0><<<grid, 256, 0, s>>>(a); break;
    case 1: zgemm_kernel<1><<<grid, 256, 0, s>>>(a); break;
    case 2: zgemm_kernel<2><<<grid, 256, 0, s>>>(a); break;
    default: throw Error(-1, "zgemm: bad precision");
  }
  PTEBD_LAUNCH_CHECK();
}

}  // namespace ptebd
