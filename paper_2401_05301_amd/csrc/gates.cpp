// Host FP64 construction of the three-site gates exp(-i h_j tau).
//
// h_j is the share of Eq. (1) on sites (j, j+1, j+2): the NNN hop (j, j+2),
// the two NN hops divided by the number of three-site windows containing
// their bond, and the on-site U and trap terms divided by the number of
// windows containing their site; summed over j it is H.  Every term conserves
// the particle number, so h_j is block diagonal in the sectors of fixed
// s1 + s2 + s3; each block is diagonalised by cyclic Jacobi rotations and the
// gate is V exp(-i w tau) V^T.
#include "gates.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace ptebd {

int windows_covering_site(int L, int s) { return std::min(s, L - 3) - std::max(0, s - 2) + 1; }
int windows_covering_bond(int L, int s) { return std::min(s, L - 3) - std::max(0, s - 1) + 1; }

static double onsite(const ModelP& m, int site, int n) {
  const double x = site + 1;  // 1-based position in the trap term
  return 0.5 * m.U * n * (n - 1) + 0.5 * m.K * (x - m.jc) * (x - m.jc) * n;
}

std::vector<double> three_site_term(const ModelP& m, int j) {
  const int d = m.d, D = d * d * d;
  std::vector<double> h((size_t)D * D, 0.0);
  auto id = [d](int a, int b, int c) { return (a * d + b) * d + c; };
  const double wl = -m.J / windows_covering_bond(m.L, j);
  const double wr = -m.J / windows_covering_bond(m.L, j + 1);
  const double wn = -m.Jnnn;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b)
      for (int c = 0; c < d; ++c) {
        const int in = id(a, b, c);
        h[(size_t)in * D + in] += onsite(m, j, a) / windows_covering_site(m.L, j) +
                                  onsite(m, j + 1, b) / windows_covering_site(m.L, j + 1) +
                                  onsite(m, j + 2, c) / windows_covering_site(m.L, j + 2);
        // hop from site y to site x (b_x^+ b_y) between occupations nx, ny
        auto hop = [&](int& nx, int& ny, double w) {
          if (ny >= 1 && nx + 1 < d) {
            const double amp = w * std::sqrt((double)(nx + 1)) * std::sqrt((double)ny);
            nx += 1; ny -= 1;
            const int out = id(a, b, c);
            nx -= 1; ny += 1;
            h[(size_t)out * D + in] += amp;
          }
        };
        hop(a, b, wl); hop(b, a, wl);   // bond (j, j+1)
        hop(b, c, wr); hop(c, b, wr);   // bond (j+1, j+2)
        hop(a, c, wn); hop(c, a, wn);   // NNN (j, j+2)
      }
  return h;
}

// Cyclic Jacobi for a dense real symmetric n x n matrix (row-major, destroyed).
// Eigenvectors returned column-wise in v (v[i*n + k] = component i of vector k).
static void jacobi_sym(std::vector<double>& a, int n, std::vector<double>& w, std::vector<double>& v) {
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  auto A = [&](int i, int k) -> double& { return a[(size_t)i * n + k]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) {
        tot += A(i, k) * A(i, k);
        if (i != k) off += A(i, k) * A(i, k);
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A(p, q);
        if (apq == 0.0) continue;
        const double tau = (A(q, q) - A(p, p)) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * akq;
          A(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * aqk;
          A(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
          v[(size_t)k * n + p] = c * vkp - s * vkq;
          v[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A(i, i);
}

SpectralGate eig_three_site(const ModelP& m, int j) {
  const int d = m.d, D = d * d * d;
  std::vector<double> h = three_site_term(m, j);
  SpectralGate g;
  g.n = D;
  g.w.assign(D, 0.0);
  g.V.assign((size_t)D * D, 0.0);
  int col = 0;
  for (int N = 0; N <= 3 * (d - 1); ++N) {
    std::vector<int> idx;
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b)
        for (int c = 0; c < d; ++c)
          if (a + b + c == N) idx.push_back((a * d + b) * d + c);
    const int n = (int)idx.size();
    if (n == 0) continue;
    std::vector<double> blk((size_t)n * n), w, v;
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) blk[(size_t)p * n + q] = h[(size_t)idx[p] * D + idx[q]];
    jacobi_sym(blk, n, w, v);
    for (int k = 0; k < n; ++k, ++col) {
      g.w[col] = w[k];
      for (int p = 0; p < n; ++p) g.V[(size_t)idx[p] * D + col] = v[(size_t)p * n + k];
    }
  }
  if (col != D) throw std::logic_error("gate sectors do not cover the three-site space");
  return g;
}

// ---- super sites (Sec. II B: every two physical sites form one site of
// dimension d^2, which makes the NNN model nearest-neighbour).  The NN hop
// inside a super site and the on-site terms of its two sites are shared by
// the gates containing that super site (one at a chain end, two in the bulk);
// the NN hop between the super sites and both NNN hops across them belong to
// gate K alone, so that the terms sum to H.
int gates_containing_super(int Ls, int K) { return std::min(K, Ls - 2) - std::max(0, K - 1) + 1; }

std::vector<double> supersite_term(const ModelP& m, int K) {
  const int d = m.d, D = d * d * d * d, Ls = m.L / 2;
  std::vector<double> h((size_t)D * D, 0.0);
  auto id = [d](const int* s) { return ((s[0] * d + s[1]) * d + s[2]) * d + s[3]; };
  const double inL = 1.0 / gates_containing_super(Ls, K), inR = 1.0 / gates_containing_super(Ls, K + 1);
  int s[4];
  for (s[0] = 0; s[0] < d; ++s[0])
    for (s[1] = 0; s[1] < d; ++s[1])
      for (s[2] = 0; s[2] < d; ++s[2])
        for (s[3] = 0; s[3] < d; ++s[3]) {
          const int in = id(s);
          h[(size_t)in * D + in] += (onsite(m, 2 * K, s[0]) + onsite(m, 2 * K + 1, s[1])) * inL +
                                    (onsite(m, 2 * K + 2, s[2]) + onsite(m, 2 * K + 3, s[3])) * inR;
          // b_x^+ b_y with amplitude w: moves one boson from position y to x
          auto hop = [&](int x, int y, double w) {
            if (s[y] >= 1 && s[x] + 1 < d) {
              const double amp = w * std::sqrt((double)(s[x] + 1)) * std::sqrt((double)s[y]);
              int t[4] = {s[0], s[1], s[2], s[3]};
              t[x] += 1;
              t[y] -= 1;
              h[(size_t)id(t) * D + in] += amp;
            }
          };
          hop(0, 1, -m.J * inL); hop(1, 0, -m.J * inL);       // inside super site K
          hop(2, 3, -m.J * inR); hop(3, 2, -m.J * inR);       // inside super site K+1
          hop(1, 2, -m.J); hop(2, 1, -m.J);                   // NN across
          hop(0, 2, -m.Jnnn); hop(2, 0, -m.Jnnn);             // NNN (2K, 2K+2)
          hop(1, 3, -m.Jnnn); hop(3, 1, -m.Jnnn);             // NNN (2K+1, 2K+3)
        }
  return h;
}

SpectralGate eig_supersite(const ModelP& m, int K) {
  const int d = m.d, D = d * d * d * d;
  std::vector<double> h = supersite_term(m, K);
  SpectralGate g;
  g.n = D;
  g.w.assign(D, 0.0);
  g.V.assign((size_t)D * D, 0.0);
  int col = 0;
  for (int N = 0; N <= 4 * (d - 1); ++N) {
    std::vector<int> idx;
    for (int i = 0; i < D; ++i) {
      int r = i, tot = 0;
      for (int q = 0; q < 4; ++q) {
        tot += r % d;
        r /= d;
      }
      if (tot == N) idx.push_back(i);
    }
    const int n = (int)idx.size();
    if (n == 0) continue;
    std::vector<double> blk((size_t)n * n), w, v;
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) blk[(size_t)p * n + q] = h[(size_t)idx[p] * D + idx[q]];
    jacobi_sym(blk, n, w, v);
    for (int k = 0; k < n; ++k, ++col) {
      g.w[col] = w[k];
      for (int p = 0; p < n; ++p) g.V[(size_t)idx[p] * D + col] = v[(size_t)p * n + k];
    }
  }
  if (col != D) throw std::logic_error("gate sectors do not cover the super-site space");
  return g;
}

void gate_matrix(const SpectralGate& g, double tau, std::vector<double>& re, std::vector<double>& im) {
  const int D = g.n;
  re.assign((size_t)D * D, 0.0);
  im.assign((size_t)D * D, 0.0);
  std::vector<double> cr(D), ci(D);
  for (int k = 0; k < D; ++k) {
    cr[k] = std::cos(g.w[k] * tau);
    ci[k] = -std::sin(g.w[k] * tau);
  }
  for (int p = 0; p < D; ++p)
    for (int k = 0; k < D; ++k) {
      const double vpk = g.V[(size_t)p * D + k];
      if (vpk == 0.0) continue;
      const double xr = vpk * cr[k], xi = vpk * ci[k];
      for (int q = 0; q < D; ++q) {
        const double vqk = g.V[(size_t)q * D + k];
        re[(size_t)p * D + q] += xr * vqk;
        im[(size_t)p * D + q] += xi * vqk;
      }
    }
}

}  // namespace ptebd
