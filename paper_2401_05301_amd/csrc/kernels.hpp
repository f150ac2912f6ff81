// Launchers of the device kernels (host side declarations).
#pragma once

#include "common.hpp"

namespace ptebd {

// C = alpha * op(A) * op(B), planar complex, row-major, batched.
//   op(A) is m x k: transA == 0 -> A(i, kk) at a[i*lda + kk];
//                   transA == 1 -> conj(A_stored(kk, i)), A_stored(kk, i) at a[kk*lda + i].
//   op(B) is k x n: transB == 0 -> B(kk, j) at b[kk*ldb + j];
//                   transB == 1 -> conj(B_stored(j, kk)) at b[j*ldb + kk].
// Optional fused scalings (device vectors; nullptr = none):
//   op(A)(i, kk) *= k_scale[kk / k_div]          (a diagonal between A and B)
//   C(i, j)      *= row_scale[i / row_div] * col_scale[j / col_div]
//   C            *= alpha * (alpha_dev ? (alpha_recip ? 1 / *alpha_dev : *alpha_dev) : 1)
// beta == 1 accumulates into C instead of overwriting it.
struct ZGemmArgs {
  int m = 0, n = 0, k = 0, batch = 1;
  const double* ar = nullptr; const double* ai = nullptr; int64_t lda = 0, sA = 0; int transA = 0;
  const double* br = nullptr; const double* bi = nullptr; int64_t ldb = 0, sB = 0; int transB = 0;
  double* cr = nullptr; double* ci = nullptr; int64_t ldc = 0, sC = 0;
  const double* k_scale = nullptr; int k_div = 1;
  const double* row_scale = nullptr; int row_div = 1;
  const double* col_scale = nullptr; int col_div = 1;
  const double* alpha_dev = nullptr; int alpha_recip = 0;
  double alpha = 1.0;
  int beta = 0;
  int herm_out = 0;   // C = X X^+ (Hermitian): accounted as 4 m^2 k flops
  const char* tag = "gemm";   // call site, for the profiler's per-site totals (a string literal)
  int tile = 0;               // FP64 tile edge: 0 = the launch rule, 64 or 128 = that tile
};

// prec: 0 = FP64 MFMA, 1 = FP32 MFMA (FP32 accumulate), 2 = split FP32 (three products).
void zgemm(const ZGemmArgs& a, int prec, hipStream_t s);

// ---------------------------------------------------------------- Jacobi SVD
// One-sided block Jacobi on the rows of X (r x c), optionally accumulating the
// row rotations into W (r x r).  Blocks of 16 rows; a round processes nb/2
// disjoint block pairs.
struct JacobiArgs {
  double* xr; double* xi; int64_t ldx;
  double* wr; double* wi; int64_t ldw;     // may be null
  int r, c;
  int nb;                                   // number of 16-row blocks, even
  int nsplit;                               // column splits of the pair Gram
  double* part;                             // [nb/2][nsplit][4][256] partial Grams
  double tol_rel, tol_abs;
  const double* tiny2;                      // device scalar: rows with |x|^2 <= *tiny2 count as zero
  unsigned int* rotated;                    // count of rotated pairs (this sweep)
  int ucols;                                // columns per update work-group
  int nuchunks;                             // update work-groups per pair
};
void jacobi_round(const JacobiArgs& a, int round, hipStream_t s);
// One round on each of `count` independent matrices (device table tab;
// gram_first / rot_first: prefix sums of nb/2 * nsplit and nb/2 * nuchunks,
// count + 1 entries, totals their last entries).  Matrices with
// active[i] == 0, or whose sweep has fewer rounds, sit the round out.
void jacobi_round_batched(const JacobiArgs* tab, const int64_t* gram_first, int64_t gram_total,
                          const int64_t* rot_first, int64_t rot_total, int count, const int* active, int round,
                          hipStream_t s);

// ------------------------------------------------- fused batches of Jacobi-route SVDs
// One matrix of a batch of one-sided Jacobi SVDs whose small steps run as one
// launch for the whole batch (fused layers).  Each step does for every
// matrix exactly what its single-matrix launcher does.
struct FusedSvdArgs {
  // staging: y = diag(rs) x (transpose = 0) or (diag(rs) x)^+ (transpose = 1), x rows x cols
  const double* xr; const double* xi; int64_t ldx;
  const double* rs; int rdiv;
  int rows, cols, transpose;
  double* yr; double* yi; int64_t ldy;
  // the Jacobi operand: the r x c rows of y (ld c), and its row norms
  int r, c;
  double* norms;
  double* wr; double* wi; int64_t ldw;      // vectors accumulated with transpose = 1 (set to the identity)
  // truncation (as select_truncate)
  int npow2, is_gram, chi_max;
  double w_max, eps;
  const double* extra_tail;
  double* lam_out; int* perm; double* inv_sig; int* info_i; double* info_d; double* ledger;
  int* kout;                                // [2]: k and the rule, contiguous over the batch
  // gather: rows perm[0..k) of g (scaled by inv_sig when gscale) into d, gc columns each
  const double* gr; const double* gi; int64_t ldg;
  int gscale, gc;
  double* dr; double* di; int64_t ldd;
};
// scale_rows_copy / conj_transpose_scaled of every matrix (max_rows, max_cols over the batch)
void fused_stage(const FusedSvdArgs* tab, int count, int max_rows, int max_cols, hipStream_t s);
// row_norms of every Jacobi operand (max_r rows at most)
void fused_row_norms(const FusedSvdArgs* tab, int count, int max_r, hipStream_t s);
// negligible_norm2 of every matrix into out[i], and the identity into the vectors of transposed ones
void fused_jacobi_prologue(const FusedSvdArgs* tab, int count, int max_r, double* out, hipStream_t s);
// select_truncate of every matrix (npow2 at most max_npow2), k and the rule also into kout
void fused_select(const FusedSvdArgs* tab, int count, int max_npow2, hipStream_t s);
// gather_rows of every matrix, k read from kout on the device (max_k over the batch)
void fused_gather(const FusedSvdArgs* tab, int count, int max_k, int max_c, hipStream_t s);

// ------------------------------------------------- two-sided Hermitian Jacobi
struct HermArgs {
  double* hr; double* hi; int64_t ldh;      // H (n x n), overwritten towards diagonal
  int n, nb;                                // nb: 16-blocks, even
  double* wr; double* wi; int64_t ldw;      // eigenvector rows (n x n) or null
  int wcols, wchunks;                       // column chunking of the W update
  double* qbuf;                             // [nb/2][2][32*32] pair rotations
  int* flag;                                // [nb/2] pair rotated this round
  unsigned int* rotated;                    // pairs rotated this sweep
  const double* tol_abs;                    // device scalar threshold
  int round;
  int inner_sweeps;                         // sweeps of the 32 x 32 pair solve per visit
};
// v[i] = sum_j v[j] for every i < n.
void share_sum(double* v, int n, hipStream_t s);
// Work-groups herm_apply uses for one round of a.
int64_t herm_apply_groups(const HermArgs& a);
// One round on each of `count` independent matrices (device table tab;
// eig_first / app_first: prefix sums of nb/2 and herm_apply_groups over the
// table, count + 1 entries; totals are their last entries).  Matrices with
// active[i] == 0, or whose sweep has fewer rounds, sit the round out.
void herm_round_batched(const HermArgs* tab, const int64_t* eig_first, int64_t eig_total, const int64_t* app_first,
                        int64_t app_total, int count, const int* active, int round, hipStream_t s);
// out[i] += number of off-diagonal entries of matrix i above *tab[i].tol_abs
// (active matrices only; max_n bounds every n; out must start at zero).
void count_above_batched(const HermArgs* tab, int count, const int* active, int max_n, unsigned int* out,
                         hipStream_t s);
// Largest |H_ij| / sqrt(max(H_ii, floor) max(H_jj, floor)) over the
// off-diagonal entries above *tol of a Hermitian PSD H (synchronises; 0 when
// none is above tol).
double offdiag_ratio(const double* hr, const double* hi, int64_t ldh, int p, const double* tol, double floor,
                     unsigned long long* ratio_bits, unsigned long long* h_ratio, hipStream_t s);
// Number of entries i < j of H (n x n) with |H_ij| > *tol (synchronises).
unsigned int count_above(const double* hr, const double* hi, int64_t ldh, int n, const double* tol,
                         unsigned int* count, unsigned int* h_count, hipStream_t s);
// H_ii = 0, i < p.
void zero_diag(double* hr, double* hi, int64_t ldh, int p, hipStream_t s);
// out[e] = sum_{i < ns} in[i * n + e] (planar, slices summed in order).
void sum_slices(const double* ir, const double* ii, int64_t n, int ns, double* orr, double* oi, hipStream_t s);
// H_ii = d[i] (real), i < p.
void set_diag(double* hr, double* hi, int64_t ldh, int p, const double* d, hipStream_t s);
// *out = c * u * sum_i |H_ii|
void herm_tol(const double* hr, int64_t ldh, int n, double c, double* out, hipStream_t s);
void herm_round(HermArgs a, int round, hipStream_t s);
// out[i] = Re H(i, i)
void herm_diag(const double* hr, int64_t ldh, int n, double* out, hipStream_t s);

// Newton-Schulz helpers on p x p planar matrices (leading dimension p).
// Scale c >= lambda_max(A) for the Newton-Schulz iteration of a Hermitian
// positive definite A (p x p): c = min(Gershgorin bound, safety * estimate)
// with the estimate from power_its power iterations (0: Gershgorin only);
// out[0] = c, out[1] = sqrt(c).  work holds 5p + 1 doubles.
void ns_scale(const double* ar, const double* ai, int p, double* work, int power_its, double safety, double* out,
              hipStream_t s);
// Y = A / *c  and  Z = I.
void ns_init(const double* ar, const double* ai, int p, const double* c, double* yr, double* yi, double* zr,
             double* zi, hipStream_t s);
// T = (3 I - P) / 2 in place; partial sums of ||T - I||_F^2 into dev[0..g),
// g returned (at most 256).
int ns_three_minus(double* pr, double* pi, int p, double* dev, hipStream_t s);

// *out = (4 u)^2 sum_i norms[i]^2: squared norm below which a row of a matrix
// with these row norms is rounding noise (u = 2^-53).
void negligible_norm2(const double* norms, int r, double* out, hipStream_t s);

// Row norms of X into norms[r] (FP64).
void row_norms(const double* xr, const double* xi, int64_t ldx, int r, int c, double* norms,
               hipStream_t s);

// Sort + truncation rule.  Inputs: vals[r] (row norms; sigma = vals, or
// sigma = sqrt(vals) if is_gram).  Writes sorted sigma/nrm for the kept values
// into lam_out[0..k), perm[0..k), inv_sig[0..k) = 1/sigma, and into info:
// info_i[0] = k; info_d[0] = nrm, info_d[1] = discarded relative weight;
// *ledger += weight.
// extra_tail (device scalar, may be null): weight of values not in vals (added
// to the total and to every tail).
void select_truncate(const double* vals, int r, int is_gram, int chi_max, double w_max, double eps,
                     double* lam_out, int* perm, double* inv_sig, int* info_i, double* info_d,
                     double* ledger, const double* extra_tail, hipStream_t s);
// Deterministic pseudo-random fill in [-1, 1) (counter hash of (seed, index)).
void fill_random(double* p, int64_t n, uint64_t seed, hipStream_t s);
// Rows of X scaled to unit 2-norm (zero rows stay zero).
void normalize_rows(double* xr, double* xi, int64_t ldx, int r, int c, double* norms, hipStream_t s);
// Y_i <- Z_i + beta_i (Y_i - theta_i Z_i) on p rows of length r, with
// beta_i = 1 / max(theta_i, |Y_i - theta_i Z_i| / gamma, damp_rel * max theta),
// and beta_i = 0 where theta_i <= zero_rel * max theta.
void damped_power_rows(const double* zr, const double* zi, double* yr, double* yi, int64_t ld, int p, int r,
                       const double* theta, double gamma, double damp_rel, double zero_rel, hipStream_t s);
// Schmidt values from an update product X = A V (rows x cols) of the
// truncated SVD of diag(rs) A = U S V^+: sigma_j = |diag(rs) X e_j| (rs[i /
// rdiv], may be null).  Writes lam[j] = sigma_j / |sigma|, *nrm = |sigma|, and
// scales X by 1 / |sigma|.  part (part_cap doubles) is scratch.
void refine_sigma(double* xr, double* xi, int64_t ldx, int rows, int cols, const double* rs, int rdiv, double* part,
                  int64_t part_cap, double* lam, double* nrm, hipStream_t s);
// out[i] = |Y_i - theta_i Z_i| (2-norm of row i, i < p, rows of length r).
void residual_norms(const double* yr, const double* yi, const double* zr, const double* zi, int64_t ld, int p, int r,
                    const double* theta, double* out, hipStream_t s);
// out[i] = 1 / sqrt(max(d[i], floor)) with floor = rel * max_j d[j] (0 if d[i] <= floor).
void inv_sqrt_clamped(const double* d, int n, double rel, double* out, hipStream_t s);
// *out = max(0, trace - sum_i vals[i]), trace = sum of diag of H.
void tail_rest(const double* hr, int64_t ldh, int n, const double* vals, int p, double* out, hipStream_t s);

// dst row i = src row perm[i] * (scale ? scale[i] : 1), i < k; planar, c columns.
void gather_rows(const double* sr, const double* si, int64_t lds, const int* perm, const double* scale,
                 int k, int c, double* dr, double* di, int64_t ldd, const int* kdev, hipStream_t s);

// ---------------------------------------------------------------- element-wise
// Y(i, j) = X(i, j) * rs[i / rdiv] (rs may be null), planar, rows x cols.
void scale_rows_copy(const double* xr, const double* xi, int64_t ldx, const double* rs, int rdiv,
                     int rows, int cols, double* yr, double* yi, int64_t ldy, hipStream_t s);
// Y(j, i) = conj(X(i, j)) * rs[i / rdiv].
void conj_transpose_scaled(const double* xr, const double* xi, int64_t ldx, const double* rs, int rdiv,
                           int rows, int cols, double* yr, double* yi, int64_t ldy, hipStream_t s);
// W = identity (r x r), planar.
void set_identity(double* wr, double* wi, int64_t ldw, int r, hipStream_t s);
// y[i] = x[i / div]^2 for i < n.
void square_expand(const double* x, int div, int n, double* y, hipStream_t s);
// Measurement helpers.
void site_densities(const double* const* br, const double* const* bi, const double* const* lam,
                    const int* chil, const int* chir, int L, int d, double* n_out, hipStream_t s);
// Correlators <O1 O2> across neighbouring sites, with O1 a creation and O2
// an annihilation operator acting on the whole site (mode 0, D = d) or on the
// first / second physical site of a super site (modes 1 / 2, D = d^2); shift
// is the change of the local index (1, d or 1).
// ks[r'] = Lambda[a]^2 sqrt(level) weights of the environment GEMM.
void op_kscale(const double* lam, int cl, int D, int d, int shift, int mode, double* ks, hipStream_t s);
// out[0..1] = sum_{y,t,c} sqrt(level(t)) conj(B(y, t - shift, c)) F(y, t, c); part: 512 doubles of scratch.
void close_op(const double* br, const double* bi, const double* fr, const double* fi, int chi, int D, int cr, int d,
              int shift, int mode, double* out, double* part, hipStream_t s);
// Per super site: (n_first, n_second, Re, Im <b+_first b_second>) into out[4 K ..].
void supersite_local(const double* const* br, const double* const* bi, const double* const* lam, const int* chil,
                     const int* chir, int Ls, int d, double* out, hipStream_t s);
// Particle-number sectors (U(1) block-sparse SVD).
// out = the block rows[0..m) x cols[0..n) of diag(rs) A (rs[r / rdiv], may be
// null): out(i, j) (trans == 0), or its conjugate transpose out(j, i)
// (trans == 1); ldo is the leading dimension of out.
void gather_block(const double* ar, const double* ai, int64_t lda, const double* rs, int rdiv, const int* rows, int m,
                  const int* cols, int n, int trans, double* outr, double* outi, int64_t ldo, hipStream_t s);
// One row copy: len values from (sr, si) into (dr, di) at positions cols[t]
// (or t when cols is null), times scale[sidx] when sidx >= 0.
struct RowCopy {
  const double* sr;
  const double* si;
  double* dr;
  double* di;
  const int* cols;
  int64_t len;
  int64_t sidx;
};
// count entries of the device table tab, one work-group each; destinations
// must not overlap.
void rows_copy(const RowCopy* tab, int count, const double* scale, hipStream_t s);
// dst[o] = src[idx[o]], o < k (dst must not alias src).
void take(const double* src, const int* idx, int k, double* dst, hipStream_t s);
void fill_zero(double* p, int64_t n, hipStream_t s);
// Cholesky factorisation of the Hermitian positive definite K (k x k,
// leading dimension k, lower triangle read) in place, K = L L^+ with L in the
// lower triangle, and X = L^-1 (k x k, leading dimension k).  t (64 k complex
// entries, planar) is scratch.  A pivot that is not positive sets *flag
// (which must start at zero).
void chol_inverse(double* kr, double* ki, int k, double* xr, double* xi, double* tr, double* ti, int* flag,
                  hipStream_t s);
// Zeroes `words` 32-bit words at p with a kernel (counters and flags: a fill
// kernel rather than hipMemsetAsync, so that the work stays plain kernel
// launches on the stream).
void fill_zero_words(void* p, int64_t words, hipStream_t s);
// *acc += sum_{i<n} slots[i], summed in index order by one thread.
void accumulate_slots(const double* slots, int n, double* acc, hipStream_t s);

}  // namespace ptebd
