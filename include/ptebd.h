/*
 * ptebd.h -- C ABI of the MI355X three-site TEBD library.
 *
 * The library evolves a matrix product state (MPS) of the 1D Bose-Hubbard
 * chain with nearest- and next-nearest-neighbour hopping and a harmonic trap
 * (Eq. (1) of the paper), starting from a charge-density-wave product state
 * (Sec. II B), by time-evolving block decimation: each Trotter layer applies
 * commuting three-site gates exp(-i h_j tau) grouped by j mod 3, contracts
 * theta, truncates it by SVD to the bond cap and updates the tensors
 * (Sec. I, Sec. II B).  Local densities and NN / NNN correlators are then
 * measured assuming orthonormality (Sec. II B; Eqs. (4), (7)).
 *
 * Conventions
 *   - Sites i = 0..L-1; bonds b = 0..L, bond b sits left of site b.
 *     Lambda_0 = Lambda_L = [1].  The trap term uses x = i + 1 (1-based), so
 *     tebd_model.jc is a 1-based position.
 *   - Stored form: B_i = Gamma_i Lambda_{i+1}, shape (chi_i, d, chi_{i+1}),
 *     row-major with chi_{i+1} fastest; complex numbers are planar (all real
 *     parts, then all imaginary parts).  Units: J = hbar = 1 (Sec. I A).
 *   - Gate g_j acts on sites (j, j+1, j+2), j = 0..L-3; group = j mod 3.
 *   - The three-site share of Eq. (1) is: the NNN hop (j, j+2) in full, each
 *     NN hop divided by the number of windows containing its bond, each
 *     on-site (U, K) term divided by the number of windows containing its
 *     site, so that the shares sum to H exactly.
 *   - Truncation (Sec. II B: bond cap chi_max, discarded-weight tolerance
 *     w_max, relative tolerance eps): singular values sorted descending,
 *     k = max(1, min(chi_max, k_w, k_eps)), k_w the smallest k with tail
 *     weight sum_{i>=k} s_i^2 <= w_max * sum_i s_i^2, k_eps = #{s_i > eps s_0};
 *     kept values renormalised to unit 2-norm; the relative tail weight is
 *     added to an FP64 ledger.  SVD across bond j+1 first, then bond j+2.
 *
 * Error behaviour: every call returns a tebd_status; no exception crosses
 * the ABI.  tebd_last_error() returns a thread-local message for the last
 * failing call on the calling thread.  EINVAL leaves the handle untouched.
 * ENOCONV (SVD did not converge within max_sweeps), and any other error
 * raised while gates are being applied (the layer is then half applied),
 * marks the handle ESTATE: later evolution and measurement calls refuse it.
 *
 * Ownership: the library owns all device memory behind an opaque handle
 * (allocated through opts.dev_alloc if given, else hipMalloc).  The caller
 * owns every host array passed in or out; host arrays are read or written
 * only during the call.  Calls on one handle must not overlap; handles are
 * independent of each other.
 */
#ifndef PTEBD_H
#define PTEBD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TEBD_OK = 0,
  TEBD_EINVAL = -1,   /* bad argument: L < 3, d < 2, chi_max < 1, group not in {0,1,2}, non-finite values */
  TEBD_ENOMEM = -2,   /* device allocation failed or footprint above budget; handle state unchanged */
  TEBD_EDEVICE = -3,  /* HIP runtime error */
  TEBD_ENOCONV = -4,  /* Jacobi SVD did not converge within max_sweeps; handle marked ESTATE */
  TEBD_ESTATE = -5    /* handle is in an error state or call not valid in its state */
} tebd_status;

/* Arithmetic of the theta assembly and gate GEMMs.  Everything else (SVD,
 * renormalisation, truncation weights, measurement) is always FP64. */
typedef enum {
  TEBD_FP64 = 0,       /* FP64 MFMA */
  TEBD_FP32 = 1,       /* FP32 MFMA, FP32 accumulation */
  TEBD_FP32_SPLIT = 2  /* hi/lo split FP32 operands, three FP32 MFMA products, FP32 accumulation */
} tebd_precision;

typedef enum {
  TEBD_SVD_JACOBI = 0,    /* one-sided block Jacobi on the rows of theta (no Gram matrix) */
  TEBD_SVD_GRAM_EIG = 1,  /* Hermitian Gram matrix + block Jacobi eigensolver; faster, squares the condition number;
                             large Gram matrices use a subspace iteration started from the Schmidt basis
                             before the gate (warm start) */
  TEBD_SVD_RANDOMIZED = 2 /* the Gram route without the warm start: every subspace iteration starts from
                             counter-hash random rows (a randomised range finder with power steps and
                             Rayleigh-Ritz, Sec. V's randomised truncation), with the same stopping rule, eps
                             floor and FP64 results; for states whose previous Schmidt basis says little
                             about the next one */
} tebd_svd;

/* Smallest relative tolerance eps (tebd_opts.trunc_rel) the Gram routes
 * accept.  The Gram matrix squares the singular values, so values below
 * about sqrt(u) s_0 (u = 2^-53) sit at its rounding level and cannot be told
 * apart from zero; eps >= 1e-6 keeps every cut the rule k_eps makes well
 * above that level.  With TEBD_SVD_GRAM_EIG or TEBD_SVD_RANDOMIZED a smaller trunc_rel is refused
 * with TEBD_EINVAL (mps_init_*, mps_footprint, tebd_serve); the one-sided
 * Jacobi route takes any eps >= 0. */
#define TEBD_GRAM_EPS_MIN 1e-6

/* Eq. (1): U/2 sum n(n-1) - J sum (b+_j b_{j+1} + h.c.) + K/2 sum (x-jc)^2 n
 *          - Jnnn sum (b+_j b_{j+2} + h.c.);  d = n_max + 1 levels per site. */
typedef struct {
  int32_t L, d;
  double U, J, Jnnn, K, jc;
} tebd_model;

typedef struct {
  int32_t chi_max;        /* bond cap (>= 1) */
  double trunc_weight;    /* w_max (>= 0) */
  double trunc_rel;       /* eps (>= 0; >= TEBD_GRAM_EPS_MIN with the Gram routes) */
  int32_t prec;           /* tebd_precision */
  int32_t svd;            /* tebd_svd */
  int32_t max_sweeps;     /* Jacobi sweep limit; <= 0 selects the default (80) */
  void* stream;           /* hipStream_t to run on; NULL = the library creates one per handle */
  void* (*dev_alloc)(size_t bytes, void* ctx);  /* optional device allocator (e.g. torch caching allocator) */
  void (*dev_free)(void* ptr, void* ctx);
  void* alloc_ctx;
  int32_t workers;        /* gate workspaces run concurrently within a layer (own stream and host
                             thread each); 0 = min(6, gates per layer), min(4, gates per layer)
                             with u1, all gates of a layer with fuse.  Device memory grows by one
                             gate workspace per worker. */
  int32_t supersite;      /* 1: the paper's super-site chain (Sec. II B): every two physical sites
                             form one site of dimension d^2 and two-site gates act on neighbouring
                             super sites, Strang A(dt/2) B(dt) A(dt/2) over gates K even / K odd.
                             The physical L must be even.  Inputs and measure_local stay physical
                             (L sites); mps_bond_dims, mps_lambda and mps_site see the L/2 super
                             sites (L/2 + 1 bonds); tebd_layer takes group 0 or 1;
                             mps_init_state is three-site only.  0: three-site gates (default). */
  int32_t u1;             /* 1: U(1) block-sparse SVDs (Sec. II B keeps the tensors in particle-number
                             sectors).  Every bond index carries the number of bosons on its left;
                             each gate's SVD is done per sector and the truncation rule runs over
                             the union of the sector spectra, so the result is the dense one.  Bond
                             indices are kept ordered by that number, then by decreasing Schmidt
                             value (mps_lambda and mps_site return this order; mps_bond_charges the
                             numbers).  Product states qualify; mps_init_state infers the numbers
                             from the non-zero entries and fails with TEBD_EINVAL when an index is
                             reached by entries of two numbers or by none.  0: dense (default). */
  int32_t fuse;           /* 1: fused layers (Sec. I: the gates of a layer are independent, and pTEBD
                             applies them together): the gates of every layer advance in lockstep
                             on the handle's stream, one per gate workspace, and their SVDs run as
                             one batched one-sided Jacobi, with one host read-back per sweep and one
                             for all truncation ranks instead of one per gate.  Results are the same
                             bit for bit; it pays where launches and host round trips dominate
                             (small chi).  Needs svd = TEBD_SVD_JACOBI, u1 = 0 and supersite = 0
                             (else TEBD_EINVAL); workers = 0 then selects one workspace per gate of
                             a layer.  0: gates spread over concurrent workers (default). */
} tebd_opts;

typedef struct tebd_mps tebd_mps;

/* Fills *opts with defaults: chi_max 64, w_max = eps = 1e-12, FP64, Jacobi. */
void tebd_opts_default(tebd_opts* opts);

/* CDW product state (Sec. II B), every bond of dimension 1.
 * first_occupied = 1: site i occupied iff i even (|1,0,1,0,...>);
 * first_occupied = 0: the opposite parity.  Reserves device memory for
 * bonds up to min(d^b, d^(L-b), chi_max) and the gate workspace. */
tebd_status mps_init_cdw(const tebd_model* model, const tebd_opts* opts,
                         int32_t first_occupied, tebd_mps** out);

/* Fock product state with occupations occ[L] (0 <= occ[i] < d). */
tebd_status mps_init_product(const tebd_model* model, const tebd_opts* opts,
                             const int32_t* occ, tebd_mps** out);

/* Arbitrary state in stored form.  chi[L+1] bond dimensions (chi[0] = chi[L] = 1,
 * each <= chi_max); B holds the sites back to back, site i as chi_i*d*chi_{i+1}
 * real parts followed by as many imaginary parts; lam holds Lambda_0..Lambda_L
 * back to back (chi[b] values each).  Host pointers, copied during the call. */
tebd_status mps_init_state(const tebd_model* model, const tebd_opts* opts,
                           const int32_t* chi, const double* B, const double* lam,
                           tebd_mps** out);

/* One commuting layer (Sec. I: the gates of a layer act on disjoint sites and
 * are applied concurrently, as in pTEBD): every gate g_j with j mod 3 ==
 * group, for a time slice tau (exp(-i h_j tau)).  Enqueued on the handle's
 * stream. */
tebd_status tebd_layer(tebd_mps* mps, int32_t group, double tau);

/* One second-order Trotter step (the appendix on numerical convergence: second-order
 * pTEBD), as the symmetric splitting over the three commuting groups:
 * layers (0, dt/2) (1, dt/2) (2, dt) (1, dt/2) (0, dt/2). */
tebd_status tebd_step(tebd_mps* mps, double dt);

/* One fourth-order step (the appendix on numerical convergence compares
 * second- with fourth-order pTEBD; the scheme it leaves open is taken as
 * Suzuki's symmetric fractal composition): five tebd_step calls of time
 * p dt, p dt, (1 - 4p) dt, p dt, p dt with p = 1 / (4 - 4^(1/3)), i.e.
 * 25 layers (15 on a super-site chain).  The middle slice runs backwards in
 * time.  Errors as tebd_step. */
tebd_status tebd_step4(tebd_mps* mps, double dt);

/* One Trotter step for n independent handles, run concurrently.  When every
 * handle has opts.fuse set, each Strang layer of all of them is one fused
 * batch on the stream of mps[0] (the gates of all handles advance in
 * lockstep and share one batched Jacobi per bond; an error then marks every
 * handle of the batch ESTATE).  Otherwise one host thread per handle issues
 * its step on the handle's own stream(s), so that their kernels overlap on
 * the device.  dt[n] per handle.  Handles must be distinct and must not have
 * been created on a shared stream.  Each handle gets exactly the result of
 * tebd_step alone. */
tebd_status tebd_step_many(tebd_mps* const* mps, int32_t n, const double* dt);

/* Local observables after the last step, FP64, synchronising the handle's stream:
 * n[L] densities; c_nn[2(L-1)] = (Re, Im) of <b+_i b_{i+1}>; c_nnn[2(L-2)] = (Re, Im)
 * of <b+_i b_{i+2}>.  Any output pointer may be NULL to skip that observable. */
tebd_status measure_local(tebd_mps* mps, double* n, double* c_nn, double* c_nnn);

/* Quasi-local observables of the experiment (Sec. II B; the quasi-local
 * densities, correlation, tunnel oscillation and visibility equations),
 * from the local n_j and C_j = <b+_j b_{j+1}> of measure_local, with the
 * lattice index j = i - centre counted from the site `centre` (0-based; the
 * centre counts as even).  out[8] = N = sum_j n_j, n_odd, n_even, Re C_even,
 * Im C_even, A, phi, nu, where n_odd/even = sum over odd/even j of n_j / N,
 * C_even = sum_{j even} C_j / N (bond j, j+1), A e^{i phi} = n_even - n_odd
 * - 2 i Im C_even (A >= 0, phi in (-pi, pi]) and nu = (1/N) sum over every
 * bond of (C_j + C_j^*).  Synchronises.  ESTATE if N is not positive. */
tebd_status measure_quasi_local(tebd_mps* mps, int32_t centre, double* out);

/* Quench: replace the Hamiltonian parameters (same L and d), keep the state. */
tebd_status mps_set_model(tebd_mps* mps, const tebd_model* model);

/* Current bond dimensions chi[L+1] (host copy; synchronises). */
tebd_status mps_bond_dims(const tebd_mps* mps, int32_t* chi);

/* Schmidt values of bond b into s[cap] in decreasing order (with opts.u1: grouped by
 * particle number, decreasing within each group); *len receives chi_b (synchronises). */
tebd_status mps_lambda(const tebd_mps* mps, int32_t bond, double* s, int32_t cap, int32_t* len);

/* With opts.u1: number of bosons left of bond `bond` for each of its indices
 * (same order as mps_lambda) into q[cap]; *len = the bond dimension.
 * TEBD_ESTATE when the handle does not track particle numbers. */
tebd_status mps_bond_charges(const tebd_mps* mps, int32_t bond, int32_t* q, int32_t cap, int32_t* len);

/* Site tensor B_i (planar: chi_i*d*chi_{i+1} reals then imaginaries) into buf[cap]. */
tebd_status mps_site(const tebd_mps* mps, int32_t site, double* buf, int64_t cap);

/* FP64 ledger: sum of relative discarded weights of all truncations so far. */
tebd_status mps_discarded_weight(const tebd_mps* mps, double* w_total);

/* Checkpoint, to resume a run later or in another process: the state in
 * stored form (bond dimensions, Schmidt values, site tensors of the chain the
 * MPS lives on) and the discarded-weight ledger, written into the host buffer
 * buf[cap] as a self-describing byte image (format tag, version, sizes, a
 * 64-bit checksum; no pointers).  *bytes receives the size of the image; with
 * buf = NULL only the size is returned.  TEBD_EINVAL when cap < *bytes;
 * TEBD_ESTATE for a handle left half applied by a failed layer.
 * Synchronises the handle and leaves it unchanged.  The Hamiltonian, the
 * options and the elapsed time are the caller's to keep. */
tebd_status mps_checkpoint(const tebd_mps* mps, void* buf, size_t cap, size_t* bytes);

/* New handle holding a checkpointed state and ledger, for the given model and
 * options: the physical L and d and opts.supersite must be those of the
 * checkpointed handle, and every bond must fit the new bond cap; with opts.u1
 * the particle numbers are inferred from the tensors as in mps_init_state.
 * Evolving it with the model and options of the original handle continues the
 * original run.  buf[len] is a host buffer read during the call.  TEBD_EINVAL
 * when the image is cut short, carries another format tag, version or
 * checksum, or does not fit model and opts. */
tebd_status mps_restore(const tebd_model* model, const tebd_opts* opts, const void* buf, size_t len,
                        tebd_mps** out);

/* Number of Jacobi sweeps used by the last SVD and their running total. */
tebd_status mps_sweep_stats(const tebd_mps* mps, int64_t* last, int64_t* total);

/* Which part of the truncation rule set k, counted over every truncation so
 * far: counts[0] the bond cap chi_max, counts[1] the weight tolerance k_w,
 * counts[2] the relative tolerance k_eps, counts[3] none (every value kept).
 * Ties are counted in that order of precedence. */
tebd_status mps_trunc_stats(const tebd_mps* mps, int64_t* counts);

/* Device bytes a handle of this model/opts reserves (state + workspace at the bond cap). */
tebd_status mps_footprint(const tebd_model* model, const tebd_opts* opts, size_t* bytes);

/* Build and upload the gates of a Strang step of size dt ahead of time, so
 * that the step itself allocates and transfers nothing.  No state change. */
tebd_status tebd_prepare(tebd_mps* mps, double dt);

/* Canonical (Vidal) form of a state loaded with mps_init_state whose B
 * tensors are right-orthonormal: identity gates are swept over j = 0..L-3, so
 * that every bond receives its exact Schmidt values given the bond to its
 * left (the handle's truncation settings apply). */
tebd_status mps_canonicalize(tebd_mps* mps);

/* Kernel classes timed by the profiler. */
typedef enum {
  TEBD_K_GEMM_FP64 = 0,   /* complex GEMM on FP64 MFMA (theta, gate, Gram, projections, updates, measurement) */
  TEBD_K_GEMM_FP32 = 1,   /* complex GEMM on FP32 MFMA (FP32 and split-FP32 theta/gate) */
  TEBD_K_HERM_EIG = 2,    /* two-sided Jacobi: 32 x 32 pair eigensolves */
  TEBD_K_HERM_APPLY = 3,  /* two-sided Jacobi: block rotations of H and W */
  TEBD_K_JAC_GRAM = 4,    /* one-sided Jacobi: pair Gram matrices */
  TEBD_K_JAC_ROTATE = 5   /* one-sided Jacobi: pair eigensolve and row rotation */
} tebd_kernel_class;

/* enable != 0: clear previous records and time every later kernel launch of
 * the handle with a pair of HIP events on the stream it runs on; 0: stop
 * recording (the totals stay readable until the next enable). */
tebd_status mps_profile(tebd_mps* mps, int32_t enable);

/* Totals over the recorded launches of one kernel class (synchronises):
 * device milliseconds, number of launches and algorithmic flops (complex
 * GEMM 8 m n k, Hermitian Gram products 4 m^2 k; 0 for the Jacobi kernels). */
tebd_status mps_profile_read(tebd_mps* mps, int32_t kclass, double* ms, int64_t* launches, double* flops);

/* Wall milliseconds, since profiling was enabled, during which at least one
 * recorded launch of the class was running (the union of the launches'
 * intervals; launches on concurrent gate workers overlap, so this can be
 * less than the summed device time of mps_profile_read).  Synchronises. */
tebd_status mps_profile_busy(tebd_mps* mps, int32_t kclass, double* busy_ms);

/* ------------------------------------------------------------------ serving
 * A stream of quench requests (CDW start, Sec. II B; Eq. (1) couplings of
 * their own; horizon = steps * dt) served concurrently.  Requests are
 * admitted first come, first served once their arrival time has passed, a
 * slot is free (max_active) and their footprint (mps_footprint) fits in what
 * the running requests leave of hbm_budget.  Each admitted request runs on
 * its own handle, stream and host thread until its horizon, so requests that
 * arrive while others run overlap with them on the device; each gets exactly
 * the result it would get alone. */
typedef struct {
  tebd_model model;
  int32_t chi_max;
  double dt;
  int32_t steps;            /* second-order Trotter steps to the horizon */
  double arrival;           /* seconds after the start of tebd_serve */
  int32_t first_occupied;   /* CDW parity, as in mps_init_cdw */
} tebd_request;

typedef struct {
  int32_t max_active;         /* concurrent requests; <= 0 selects 8 */
  double hbm_budget;          /* device bytes the admitted requests may reserve; <= 0: 85% of the free memory */
  int32_t prec, svd;          /* tebd_precision, tebd_svd for every request */
  double trunc_weight, trunc_rel;
  int32_t workers_per_request;  /* gate workers of each request's handle; <= 0 selects 1 */
  int32_t measure_every;      /* measure_local every this many steps as well (0: only at the horizon) */
  int32_t u1;                 /* tebd_opts.u1 for every request (0 or 1) */
  int32_t batched;            /* 1: continuous batching -- one scheduler thread steps every admitted
                                 request together, each Strang layer of all of them one fused batch
                                 (tebd_step_many with tebd_opts.fuse); arrivals join and finished
                                 requests leave between steps.  Needs svd = TEBD_SVD_JACOBI and
                                 u1 = 0; workers_per_request <= 0 then gives each request one gate
                                 workspace per gate of a layer.  A failing step fails every request
                                 in that batch.  0: a thread per request (default). */
} tebd_serve_opts;

typedef struct {
  double arrival, admitted, finished;   /* seconds after the start of tebd_serve */
  double discarded_weight;             /* FP64 ledger at the horizon */
  int64_t gate_updates;                /* three-site gate updates performed */
  int32_t status;                      /* tebd_status of this request */
} tebd_serve_result;

/* Serves req[n]; fills res[n] and, for request i in order, the observables
 * at its horizon (as measure_local) at offsets sum_{k<i} L_k in n_out,
 * sum_{k<i} 2(L_k-1) in c_nn and sum_{k<i} 2(L_k-2) in c_nnn (any output may
 * be NULL).  Returns after every request has finished; EINVAL/ENOMEM before
 * anything runs if a request is invalid or larger than the budget alone,
 * else the first failing request's status (the others still run). */
tebd_status tebd_serve(const tebd_request* req, int32_t n, const tebd_serve_opts* opts, tebd_serve_result* res,
                       double* n_out, double* c_nn, double* c_nnn);

/* Block until all work enqueued on the handle has finished. */
tebd_status mps_sync(tebd_mps* mps);

/* Release the handle and its device memory.  NULL is accepted. */
tebd_status mps_free(tebd_mps* mps);

/* Thread-local message of the last failing call ("" if none). */
const char* tebd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PTEBD_H */
