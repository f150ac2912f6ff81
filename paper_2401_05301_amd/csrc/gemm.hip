// Complex planar GEMM on the gfx950 matrix cores.
//
// A work-group computes a 64 x 64 tile of C with four waves or (FP64, large
// C) a 128 x 128 tile with eight; each wave owns a block of MFMA tiles of
// 16 x 16.  The complex product is four real products (Cr += Ar Br - Ai Bi,
// Ci += Ar Bi + Ai Br), so both rounding errors stay symmetric.  K is walked
// in slabs of 16 through two LDS buffers; tiles are ordered so that each XCD
// works on a compact block of them.  Precisions:
//   FP64  : v_mfma_f64_16x16x4_f64
//   FP32  : operands rounded to FP32, v_mfma_f32_16x16x4_f32, FP32 accumulation
//   SPLIT : x = hi + lo with hi = fl32(x), lo = fl32(x - hi); products
//           hi*hi + hi*lo + lo*hi, FP32 accumulation.
#include <type_traits>

#include "kernels.hpp"
#include "profile.hpp"

namespace ptebd {

namespace {

constexpr int PAD = 1;

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

template <int PREC, int KB, int LD>
__device__ __forceinline__ void put(typename Traits<PREC>::T (*s)[KB][LD], int kk, int r, double v) {
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

// Work-groups are dispatched round-robin over the eight XCDs of the chip
// (work-group b runs on XCD b mod 8), and each XCD has its own L2.  The
// linear work-group index is mapped so that XCD x receives one contiguous
// range of the logical tile order: the tiles that run together on one XCD
// then share operand panels in its L2.  The map is a bijection of [0, T).
__device__ __forceinline__ int xcd_logical(int bid, int T) {
  constexpr int kXcd = 8;
  const int q = T / kXcd, rem = T % kXcd;
  const int x = bid % kXcd, i = bid / kXcd;
  return x * q + min(x, rem) + i;
}

// Logical tile t of a rows x cols tile grid in groups of kGroup tile rows:
// consecutive tiles walk down a group's rows first, then along its columns,
// so that a run of consecutive tiles covers a block of about kGroup x
// (run / kGroup) tiles and re-reads few A and B panels.
__device__ __forceinline__ void grouped_tile(int t, int rows, int cols, int& tr, int& tc) {
  constexpr int kGroup = 8;
  const int per_group = kGroup * cols;
  const int grp = t / per_group;
  const int first = grp * kGroup;
  const int gsize = min(rows - first, kGroup);
  const int u = t - grp * per_group;
  tr = first + u % gsize;
  tc = u / gsize;
}

// Tile BM x BN per work-group of WM x WN waves; each wave owns a
// (BM/WM) x (BN/WN) block as TM x TN MFMA tiles of 16 x 16.  K advances in
// slabs of BK through two LDS buffers: while the waves multiply slab t out
// of one buffer, the global loads of slab t+1 are in flight into registers
// and are then staged into the other buffer, so one barrier per slab
// separates the two.
template <int PREC, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void zgemm_kernel(ZGemmArgs g) {
  using Tr = Traits<PREC>;
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  constexpr int NP = Tr::NPART;
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
  constexpr int RA = BM * BK / NT, RB = BN * BK / NT;   // loads per thread per slab
  __shared__ T As_r[2][NP][BK][BM + PAD], As_i[2][NP][BK][BM + PAD];
  __shared__ T Bs_r[2][NP][BK][BN + PAD], Bs_i[2][NP][BK][BN + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t bz = blockIdx.z;
  int tile_r, tile_c;
  if (g.herm_out) {
    // lower-triangular tiles only (tile_c <= tile_r), linearised by rows
    const int T_ = ceil_div(g.m, BM);
    const int t = xcd_logical(blockIdx.x, T_ * (T_ + 1) / 2);
    int ty = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((ty + 1) * (ty + 2) / 2 <= t) ++ty;
    while (ty * (ty + 1) / 2 > t) --ty;
    tile_r = ty;
    tile_c = t - ty * (ty + 1) / 2;
  } else {
    const int rows = ceil_div(g.m, BM), cols = ceil_div(g.n, BN);
    grouped_tile(xcd_logical(blockIdx.x, rows * cols), rows, cols, tile_r, tile_c);
  }
  const int row0 = tile_r * BM, col0 = tile_c * BN;
  const double* Ar = g.ar + bz * g.sA;
  const double* Ai = g.ai + bz * g.sA;
  const double* Br = g.br + bz * g.sB;
  const double* Bi = g.bi + bz * g.sB;

  Acc accr[TM][TN], acci[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      accr[a][b] = Acc{0, 0, 0, 0};
      acci[a][b] = Acc{0, 0, 0, 0};
    }

  // Element e = tid + NT rep of a slab: k fastest when the operand is
  // contiguous in k, else the row (column) index fastest, so that
  // neighbouring lanes read neighbouring addresses.  Every load is
  // unconditional, from an index clamped into the matrix, so that all of a
  // slab's loads are in flight together; elements outside the matrix are
  // zeroed (and k-scaled) when staged.
  double ra_r[RA], ra_i[RA], rb_r[RB], rb_i[RB], rks[RA];
  int slab_k0 = 0;
  auto load = [&](int k0) {
    slab_k0 = k0;
#pragma unroll
    for (int rep = 0; rep < RA; ++rep) {
      const int e = tid + NT * rep;
      const int kk = g.transA ? e / BM : e % BK;
      const int i = min(row0 + (g.transA ? e % BM : e / BK), g.m - 1);
      const int kg = min(k0 + kk, g.k - 1);
      const int64_t o = g.transA ? (int64_t)kg * g.lda + i : (int64_t)i * g.lda + kg;
      ra_r[rep] = Ar[o];
      ra_i[rep] = Ai[o];
      rks[rep] = g.k_scale ? g.k_scale[kg / g.k_div] : 1.0;
    }
#pragma unroll
    for (int rep = 0; rep < RB; ++rep) {
      const int e = tid + NT * rep;
      const int kk = g.transB ? e % BK : e / BN;
      const int j = min(col0 + (g.transB ? e / BK : e % BN), g.n - 1);
      const int kg = min(k0 + kk, g.k - 1);
      const int64_t o = g.transB ? (int64_t)j * g.ldb + kg : (int64_t)kg * g.ldb + j;
      rb_r[rep] = Br[o];
      rb_i[rep] = Bi[o];
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int rep = 0; rep < RA; ++rep) {
      const int e = tid + NT * rep;
      const int kk = g.transA ? e / BM : e % BK;
      const int i = g.transA ? e % BM : e / BK;
      const bool ok = row0 + i < g.m && slab_k0 + kk < g.k;
      const double sc = ok ? rks[rep] : 0.0;
      put<PREC, BK, BM + PAD>(As_r[buf], kk, i, ra_r[rep] * sc);
      put<PREC, BK, BM + PAD>(As_i[buf], kk, i, (g.transA ? -ra_i[rep] : ra_i[rep]) * sc);
    }
#pragma unroll
    for (int rep = 0; rep < RB; ++rep) {
      const int e = tid + NT * rep;
      const int kk = g.transB ? e % BK : e / BN;
      const int j = g.transB ? e / BK : e % BN;
      const bool ok = col0 + j < g.n && slab_k0 + kk < g.k;
      put<PREC, BK, BN + PAD>(Bs_r[buf], kk, j, ok ? rb_r[rep] : 0.0);
      put<PREC, BK, BN + PAD>(Bs_i[buf], kk, j, ok ? (g.transB ? -rb_i[rep] : rb_i[rep]) : 0.0);
    }
  };
  // The four real products of each k step are issued product by product
  // over all of the wave's tiles, so that the two updates of one
  // accumulator are TM * TN matrix instructions apart.
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T ar[NP][TM], ai[NP][TM], br[NP][TN], bi[NP][TN];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int t = 0; t < TM; ++t) {
          ar[p][t] = As_r[buf][p][kr][wm * (BM / WM) + t * 16 + (lane & 15)];
          ai[p][t] = As_i[buf][p][kr][wm * (BM / WM) + t * 16 + (lane & 15)];
        }
#pragma unroll
        for (int t = 0; t < TN; ++t) {
          br[p][t] = Bs_r[buf][p][kr][wn * (BN / WN) + t * 16 + (lane & 15)];
          bi[p][t] = Bs_i[buf][p][kr][wn * (BN / WN) + t * 16 + (lane & 15)];
        }
      }
      if constexpr (PREC != 2) {
        T nai[TM];
#pragma unroll
        for (int a = 0; a < TM; ++a) nai[a] = -ai[0][a];
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) accr[a][b] = mfma(ar[0][a], br[0][b], accr[a][b]);
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) acci[a][b] = mfma(ar[0][a], bi[0][b], acci[a][b]);
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) accr[a][b] = mfma(nai[a], bi[0][b], accr[a][b]);
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) acci[a][b] = mfma(ai[0][a], br[0][b], acci[a][b]);
      } else {
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) {
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
  };

  const int nslab = ceil_div(g.k, BK);
  load(0);
  stage(0);
  __syncthreads();
  for (int t = 0; t < nslab; ++t) {
    const int cur = t & 1;
    if (t + 1 < nslab) load((t + 1) * BK);
    compute(cur);
    // the other buffer was last read in iteration t - 1, before the barrier
    if (t + 1 < nslab) stage(cur ^ 1);
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
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = row0 + wm * (BM / WM) + a * 16 + (PREC == 0 ? (lane >> 4) + 4 * e : 4 * (lane >> 4) + e);
        const int j = col0 + wn * (BN / WN) + b * 16 + (lane & 15);
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

template <int PREC, int BM, int BN, int BK, int WM, int WN>
void launch(const ZGemmArgs& a, hipStream_t s) {
  const int64_t rows = ceil_div(a.m, BM), cols = ceil_div(a.n, BN);
  const int64_t T = a.herm_out ? rows * (rows + 1) / 2 : rows * cols;
  if (T > (int64_t)1 << 30) throw Error(-1, "zgemm: too many tiles");
  dim3 grid((unsigned)T, 1, a.batch);
  if (grid.z > 65535) throw Error(-1, "zgemm: grid too large");
  zgemm_kernel<PREC, BM, BN, BK, WM, WN><<<grid, 64 * WM * WN, 0, s>>>(a);
}

// 128 x 128 launches run one work-group per CU at a time (256 CUs): use them
// for at least one full wave and a last wave at least half full.
bool wide_tiles_pay(int64_t t) {
  if (t < 256) return false;
  const int64_t rest = t % 256;
  return t >= 1024 || rest == 0 || rest >= 128;
}

// Number of work-groups a launch with BM x BN tiles would have.
int64_t tiles(const ZGemmArgs& a, int bm, int bn) {
  if (a.herm_out) {
    const int64_t T = ceil_div(a.m, bm);
    return T * (T + 1) / 2 * a.batch;
  }
  return (int64_t)ceil_div(a.m, bm) * ceil_div(a.n, bn) * a.batch;
}

}  // namespace

void zgemm(const ZGemmArgs& a, int prec, hipStream_t s) {
  if (a.m <= 0 || a.n <= 0 || a.batch <= 0) return;
  if (a.k <= 0) throw Error(-1, "zgemm: k must be positive");
  if (a.tile != 0 && a.tile != 64 && a.tile != 128) throw Error(-1, "zgemm: tile must be 0, 64 or 128");
  if (a.herm_out) {
    // C = X X^+ is Hermitian: only tiles on or below the diagonal are computed
    if (a.m != a.n || a.beta || a.col_scale != a.row_scale || a.col_div != a.row_div)
      throw Error(-1, "zgemm: Hermitian output needs a square, overwritten, symmetrically scaled C");
  }
  // algorithmic work: a Hermitian Gram product counts as a rank-k update
  const double flops = a.herm_out ? 4.0 * a.m * a.m * (double)a.k * a.batch
                                  : 8.0 * a.m * (double)a.n * a.k * a.batch;
  ProfScope ps(prec == 0 ? K_GEMM_FP64 : K_GEMM_FP32, flops, s, a.tag);
  switch (prec) {
    case 0: {
      // 128 x 128 tiles halve the operand traffic per flop; they pay off
      // when the launch fills the chip with them without a thin last wave
      if (a.tile == 128 || (a.tile == 0 && wide_tiles_pay(tiles(a, 128, 128))))
        launch<0, 128, 128, 16, 4, 2>(a, s);
      else
        launch<0, 64, 64, 16, 2, 2>(a, s);
      break;
    }
    case 1: launch<1, 64, 64, 16, 2, 2>(a, s); break;
    case 2: launch<2, 64, 64, 16, 2, 2>(a, s); break;
    default: throw Error(-1, "zgemm: bad precision");
  }
  PTEBD_LAUNCH_CHECK();
}

}  // namespace ptebd
