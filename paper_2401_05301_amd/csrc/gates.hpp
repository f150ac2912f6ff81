// Host FP64 gate builder (see gates.cpp).
#pragma once

#include <vector>

namespace ptebd {

struct ModelP {
  int L, d;
  double U, J, Jnnn, K, jc;
};

struct SpectralGate {
  int n = 0;                 // d^3
  std::vector<double> w;     // eigenvalues of h_j
  std::vector<double> V;     // V[i*n + k]: component i of eigenvector k (real)
};

int windows_covering_site(int L, int s);
int windows_covering_bond(int L, int s);
std::vector<double> three_site_term(const ModelP& m, int j);   // d^3 x d^3, row-major
SpectralGate eig_three_site(const ModelP& m, int j);
// Super-site chain (two physical sites per super site, m.L even): the
// two-super-site term on super sites (K, K+1) = physical sites 2K..2K+3,
// d^4 x d^4 row-major, and its spectral decomposition.
int gates_containing_super(int Ls, int K);
std::vector<double> supersite_term(const ModelP& m, int K);
SpectralGate eig_supersite(const ModelP& m, int K);
void gate_matrix(const SpectralGate& g, double tau, std::vector<double>& re, std::vector<double>& im);

}  // namespace ptebd
