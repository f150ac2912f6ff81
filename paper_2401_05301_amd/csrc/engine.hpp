// MPS store and gate-update driver (host side).
#pragma once

#include <map>
#include <utility>
#include <vector>

#include "../../include/ptebd.h"
#include "common.hpp"
#include "gates.hpp"
#include "kernels.hpp"

struct tebd_mps {
  ptebd::ModelP model{};
  tebd_opts opts{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int L = 0, d = 0, chi_max = 0;
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
  unsigned int* h_counter = nullptr;  // pinned host mirrors
  int* h_info = nullptr;

  std::vector<void*> allocs;
  std::vector<ptebd::SpectralGate> spectra;          // per j
  std::map<std::pair<int, double>, std::pair<double*, double*>> gates;  // (j, tau) -> device G

  bool failed = false;
  int64_t last_sweeps = 0, total_sweeps = 0;
};

namespace ptebd {

struct Sizes {
  std::vector<int> cap;
  int64_t site_elems = 0, lam_elems = 0;
  int64_t T1 = 0, psi = 0, X2 = 0, G = 0, W = 0, V1h = 0, meas_sq = 0, meas_rect = 0, vec = 0, part = 0;
  int64_t gates = 0;
  size_t bytes() const;
};

Sizes plan_sizes(int L, int d, int chi_max);
void mps_allocate(tebd_mps* M);
void mps_release(tebd_mps* M);
void upload_product(tebd_mps* M, const int* occ);
void upload_state(tebd_mps* M, const int* chi, const double* B, const double* lam);
void set_model(tebd_mps* M, const ModelP& m);
void layer(tebd_mps* M, int group, double tau);
void measure(tebd_mps* M, double* n, double* cnn, double* cnnn);

struct SvdIn {
  const double* ar;
  const double* ai;
  int64_t lda;
  int m, n;
  const double* rs;   // row scale of the input (Lambda), may be null
  int rdiv;
};
// Truncated SVD of diag(rs) A with the handle's settings (see engine.cpp).
int svd_trunc(tebd_mps* M, const SvdIn& in, double* lam_out, double* vhr, double* vhi, int slot, tebd_mps::Z xbuf);
void* dev_alloc(tebd_mps* M, size_t bytes);

}  // namespace ptebd
