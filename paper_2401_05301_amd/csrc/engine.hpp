// MPS store and gate-update driver (host side).
#pragma once

#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/ptebd.h"
#include "common.hpp"
#include "gates.hpp"
#include "kernels.hpp"
#include "profile.hpp"

namespace ptebd {
// Tile shapes of the theta and gate products chosen by measurement, for the
// whole process: for every (device, m, n, k, batch) seen, the faster of the
// 64 x 64 and 128 x 128 FP64 tiles, timed on the real operands at first use.
struct TileTuner {
  std::mutex mu;
  std::map<std::array<int64_t, 5>, int> best;
  int64_t shapes_tuned = 0, launches_128 = 0, launches_64 = 0;
};
TileTuner& tile_tuner();
}  // namespace ptebd

struct tebd_mps {
  ptebd::ModelP model{};
  tebd_opts opts{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int L = 0, d = 0, chi_max = 0;    // sites and local dimension of the chain the MPS lives on
  bool super = false;               // super-site chain: L = phys_L / 2 sites of dimension d = pd^2
  int phys_L = 0, pd = 0;           // physical sites and their local dimension
  // Particle-number sectors (opts.u1): bosons left of every bond index
  // (b = 0..L, chi[b] entries each; held by the state) and bosons of every
  // local level (d entries).
  bool u1 = false;
  std::vector<std::vector<int>> q;
  std::vector<int> qs;
  std::vector<int> cap;   // bond capacity, b = 0..L
  std::vector<int> chi;   // current bond dimension, b = 0..L (host mirror)

  // device state
  std::vector<double*> Br, Bi;   // site tensors (planar)
  std::vector<double*> lam;      // Schmidt values per bond
  double* ledger = nullptr;      // discarded weight (FP64)

  // device pointer tables for measurement
  double** d_br = nullptr;
  double** d_bi = nullptr;
  double** d_lam = nullptr;
  int* d_chi = nullptr;

  // workspace (planar complex buffers: re, im)
  struct Z { double* re = nullptr; double* im = nullptr; };
  Z T1, psi, psip, X2, G, W, V1h;
  Z sZ, sY, sZ2, sY2, sH, sW;   // subspace iteration: bases (p x r) and p x p blocks
  Z nY, nZ, nY2, nZ2;           // Newton-Schulz iterates (p x p)
  double* ns_part = nullptr;    // Newton-Schulz residual partial sums (256)
  double* h_part = nullptr;     // pinned host mirror of ns_part
  unsigned long long* ratio_bits = nullptr;   // largest relative coupling of a Rayleigh matrix (bits of a double)
  unsigned long long* h_ratio = nullptr;      // pinned host mirror
  double* pwork = nullptr;      // Newton-Schulz scale: row sums and power-iteration vectors (5p + 1)
  int sub_p = 0;                // subspace width reserved (0: not reserved)
  int sub_r = 0;                // row length reserved for the subspace bases
  int64_t g_cap = 0;            // entries of the Gram workspaces G and W
  int* flags = nullptr;         // per block pair flags of the Hermitian Jacobi
  Z E, F, F2, F3;
  double* ks = nullptr;
  double* norms = nullptr;
  double* inv_sig = nullptr;
  double* sq = nullptr;
  int* perm = nullptr;
  double* part = nullptr;
  int64_t part_cap = 0;
  int* info_i = nullptr;       // [4]
  double* info_d = nullptr;    // [8]: nrm1, w1, nrm2, w2, ...
  unsigned int* counter = nullptr;
  double* meas = nullptr;      // n[L], C[2(L-1)], D[2(L-2)]
  double* hop_part = nullptr;  // partial sums of the correlator closes (512)
  unsigned int* h_counter = nullptr;  // pinned host mirrors
  int* h_info = nullptr;

  std::vector<void*> allocs;
  std::vector<ptebd::SpectralGate> spectra;          // per j
  // Device gates: kGateSlots buffers per window j, each holding G_j(tau) for
  // one tau, reused least recently used first (set_model invalidates them).
  struct GateSlot {
    double tau = 0.0;
    bool valid = false;
    uint64_t used = 0;
    double* re = nullptr;
    double* im = nullptr;
  };
  std::vector<std::vector<GateSlot>> gates;
  uint64_t gate_clock = 0;

  bool failed = false;
  int64_t last_sweeps = 0, total_sweeps = 0;
  int64_t rule_counts[4] = {0, 0, 0, 0};   // truncations set by chi_max, k_w, k_eps, none (this workspace)

  ptebd::Profiler prof;   // kernel timings while profiling is enabled
  bool prof_on = false;

  // Gate workspaces.  The gates of one layer act on disjoint sites, so they
  // are spread over workers, each with its own buffers, stream and host
  // thread; worker 0 runs on the handle's stream.  A worker is a tebd_mps
  // that holds workspace only (its parent holds the state).
  std::vector<tebd_mps*> workers;
  tebd_mps* parent = nullptr;
  double* wslots = nullptr;   // discarded weight of each gate of the current layer (device, L)

  // Sector tables of one U(1) SVD (workers only): row and column lists and
  // the output order on the device, the row-copy table, the projected rows.
  int* u_idx = nullptr;
  int64_t u_idx_cap = 0;
  ptebd::RowCopy* u_tab = nullptr;
  int64_t u_tab_cap = 0;
  Z uv;
  std::vector<int> h_idx, h_perm, h_order;
  std::vector<ptebd::RowCopy> h_tab;
  void* u_batch = nullptr;        // batched Jacobi tables of the sector eigenproblems
  int64_t u_batch_cap = 0;        // bytes
  int64_t flags_cap = 0;          // entries of flags
  // Fused layers (opts.fuse): descriptor table of a batch of SVDs (device and
  // pinned host staging, kFusedMax entries) and their truncation ranks.
  ptebd::FusedSvdArgs* f_tab = nullptr;
  ptebd::FusedSvdArgs* h_ftab = nullptr;
  int* f_k = nullptr;
  int* h_fk = nullptr;
  std::vector<ptebd::HermArgs> h_herm;
  std::vector<int64_t> h_first;
  std::vector<int> h_active;
  std::vector<unsigned int> h_counts;
};

namespace ptebd {

// Time slices whose gates stay resident per window (a Strang step needs
// one per window, a fourth-order step two, canonicalisation one more).
constexpr int kGateSlots = 4;

struct Sizes {
  std::vector<int> cap;
  int64_t site_elems = 0, lam_elems = 0;
  int64_t T1 = 0, psi = 0, X2 = 0, G = 0, W = 0, V1h = 0, meas_sq = 0, meas_rect = 0, vec = 0, part = 0;
  int64_t sub_p = 0, sub_r = 0;   // subspace iteration width and row length
  int64_t gates = 0;
  int64_t uv = 0, idx = 0;         // U(1) SVD: projected rows (k x n) and sector lists (m + n)
  size_t bytes(int workers, bool u1 = false, bool fuse = false) const;
};

// Number of gate workers of a handle: opts.workers if positive, else 6 (4 with
// particle-number sectors, one per gate of a layer with fused layers), at
// most the number of gates in a layer (L sites of the chain the MPS lives
// on; two-site gates on a super-site chain).
int auto_workers(int L, int requested, bool super = false, bool u1 = false, bool fuse = false);
// Device bytes of the batched Jacobi tables of a fused-layer workspace on L sites.
int64_t fused_table_bytes(int L);
// Largest batch of SVDs one fused step launches together.
constexpr int kFusedMax = 256;

Sizes plan_sizes(int L, int d, int chi_max);
// Sizes of a super-site chain of Ls sites of dimension D (two-site gates).
Sizes plan_sizes2(int Ls, int D, int chi_max);
// Width of the subspace used for the top-k eigenpairs of an r x r Gram
// matrix when keeping at most chi_max values (0: solve the whole matrix).
int subspace_width(int r, int chi_max);
// The same for a given number of values to keep, with the narrow or the wide
// oversampling (0 where the whole matrix is solved directly).
int subspace_width_keep(int r, int keep, bool wide);
void mps_allocate(tebd_mps* M);
void mps_release(tebd_mps* M);
void upload_product(tebd_mps* M, const int* occ);
void upload_state(tebd_mps* M, const int* chi, const double* B, const double* lam);
void set_model(tebd_mps* M, const ModelP& m);
void layer(tebd_mps* M, int group, double tau);
// Layer `group` of every handle in Ms (time slice taus[h] for handle h) as one
// fused batch on the stream of Ms[0]: every handle has opts.fuse set (three-
// site chain, Jacobi route).  Each handle's result is the one layer() gives;
// an error marks every handle of the batch failed.
void layers_many(const std::vector<tebd_mps*>& Ms, int group, const std::vector<double>& taus);
// Sweep of identity gates j = 0..L-3: brings a right-orthonormal state into
// the canonical form with exact Schmidt values (up to truncation).
void canonicalize(tebd_mps* M);
// Sweeps of the last SVD (max over workers) and their running total.
void sweep_stats(const tebd_mps* M, int64_t* last, int64_t* total);
// Truncations of the handle by the part of the rule that set k (summed over workers).
void trunc_stats(const tebd_mps* M, int64_t* counts);
// Build and upload the gates of the given group and time slice (no state change).
void prepare_gates(tebd_mps* M, int group, double tau);
void measure(tebd_mps* M, double* n, double* cnn, double* cnnn);

// Starting rows for the subspace iteration of the Gram route: the singular
// vectors of the state before the gate, on the side the Gram matrix lives on.
struct WarmStart {
  int kind = 0;                 // 0 none, 1 rows = conj((diag(rs) S)^T), 2 rows = S
  const double* sr = nullptr;   // source S (src_rows x src_cols), leading dimension ld
  const double* si = nullptr;
  int64_t ld = 0;
  int src_rows = 0, src_cols = 0;
  const double* rs = nullptr;
  int rdiv = 1;
};

struct SvdIn {
  const double* ar;
  const double* ai;
  int64_t lda;
  int m, n;
  const double* rs;   // row scale of the input (Lambda), may be null
  int rdiv;
  bool prefer_right = false;   // Gram route: use A^+ A when n <= m (not only n < m)
  WarmStart warm;
};
// Truncated SVD of diag(rs) A with the handle's settings (see engine.cpp).
int svd_trunc(tebd_mps* M, const SvdIn& in, double* lam_out, double* vhr, double* vhi, int slot, tebd_mps::Z xbuf);
// The same for an A whose rows and columns carry particle numbers rq[m] and
// cq[n], A(r, c) = 0 unless rq[r] == cq[c]: every sector is decomposed on its
// own and the truncation rule is applied to the union of their spectra.  The
// kept rows of V^+ (and kept_q, their particle numbers) are ordered by
// particle number, then by decreasing singular value; lam_out likewise.
int svd_trunc_u1(tebd_mps* M, const SvdIn& in, const std::vector<int>& rq, const std::vector<int>& cq,
                 double* lam_out, double* vhr, double* vhi, int slot, tebd_mps::Z xbuf, std::vector<int>& kept_q);
// Particle numbers of every bond index of an uploaded state, inferred from
// the non-zero entries of its tensors (host copies in mps_init_state
// layout); throws an EINVAL Error when an index is reached by entries of two
// numbers or by none.
std::vector<std::vector<int>> infer_charges(const tebd_mps* M, const int* chi, const double* B);
void* dev_alloc(tebd_mps* M, size_t bytes);

}  // namespace ptebd
