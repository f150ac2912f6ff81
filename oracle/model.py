"""Eq. (1) of the paper, its split into three-site terms, and the gates.

Units: J = hbar = 1 (Sec. I A), so a gate for a time slice tau is
exp(-i h tau) with tau in units of hbar/J.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from workloads import Model


def boson_ops(d: int):
    """Annihilator b and number operator n on one site, truncated at
    n_max = d - 1 (Sec. II B: local dimension d = n_max + 1).

    <n-1| b |n> = sqrt(n); b^+ |n_max> = 0, which keeps particle number
    exactly conserved by every hopping term.
    """
    b = np.zeros((d, d))
    for n in range(1, d):
        b[n - 1, n] = np.sqrt(n)
    num = np.diag(np.arange(d, dtype=np.float64))
    return b, num


def onsite_energy(m: Model, i: int) -> np.ndarray:
    """U/2 n(n-1) + K/2 (x - j_c)^2 n for 0-based site i, x = i + 1 (Eq. (1))."""
    _, num = boson_ops(m.d)
    x = i + 1
    eye = np.eye(m.d)
    return 0.5 * m.U * num @ (num - eye) + 0.5 * m.K * (x - m.centre()) ** 2 * num


def gates_covering_site(L: int, s: int) -> int:
    """Number of three-site windows (j, j+1, j+2), 0 <= j <= L-3, containing site s."""
    return min(s, L - 3) - max(0, s - 2) + 1


def gates_covering_bond(L: int, s: int) -> int:
    """Number of three-site windows containing the bond (s, s+1)."""
    return min(s, L - 3) - max(0, s - 1) + 1


def kron3(a, b, c):
    return np.kron(a, np.kron(b, c))


def three_site_term(m: Model, j: int) -> np.ndarray:
    """h_j on sites (j, j+1, j+2), a d^3 x d^3 Hermitian matrix.

    Index order (s_j, s_{j+1}, s_{j+2}) with s_j slowest.  Each term of
    Eq. (1) is shared equally among the windows that contain it: the
    NNN hop (j, j+2) belongs to window j alone, an NN hop on bond (s, s+1)
    is divided by the number of windows containing that bond, and the
    on-site U and trap terms of site s by the number of windows containing
    site s.  Summed over j = 0..L-3 this reproduces H exactly.
    """
    L, d = m.L, m.d
    if L < 3:
        raise ValueError("three-site gates need L >= 3")
    b, _ = boson_ops(d)
    bd = b.T
    eye = np.eye(d)
    h = np.zeros((d ** 3, d ** 3))
    # NNN hopping, Eq. (1) last term
    h += -m.Jnnn * (kron3(bd, eye, b) + kron3(b, eye, bd))
    # NN hopping on the two bonds inside the window
    hop_left = -m.J * (kron3(bd, b, eye) + kron3(b, bd, eye))
    hop_right = -m.J * (kron3(eye, bd, b) + kron3(eye, b, bd))
    h += hop_left / gates_covering_bond(L, j)
    h += hop_right / gates_covering_bond(L, j + 1)
    # on-site interaction and trap
    for pos in range(3):
        s = j + pos
        ops = [eye, eye, eye]
        ops[pos] = onsite_energy(m, s)
        h += kron3(*ops) / gates_covering_site(L, s)
    return h


def gate(m: Model, j: int, tau: float) -> np.ndarray:
    """G_j(tau) = exp(-i h_j tau) via the spectral decomposition of h_j."""
    w, v = np.linalg.eigh(three_site_term(m, j))
    return (v * np.exp(-1j * w * tau)) @ v.conj().T


def full_hamiltonian(m: Model) -> sp.csr_matrix:
    """Eq. (1) on the whole chain as a sparse d^L x d^L matrix.

    Built directly from the equation (not from the three-site split) so
    that the split can be checked against it.  Site 0 is the slowest index.
    """
    L, d = m.L, m.d
    b, num = boson_ops(d)
    bd = b.T
    I = sp.identity(d, format="csr")

    def embed(ops):
        # ops: dict site -> d x d matrix
        out = None
        for s in range(L):
            o = sp.csr_matrix(ops[s]) if s in ops else I
            out = o if out is None else sp.kron(out, o, format="csr")
        return out

    H = sp.csr_matrix((d ** L, d ** L), dtype=np.float64)
    for s in range(L):
        H = H + embed({s: onsite_energy(m, s)})
    for s in range(L - 1):
        H = H - m.J * (embed({s: bd, s + 1: b}) + embed({s: b, s + 1: bd}))
    for s in range(L - 2):
        H = H - m.Jnnn * (embed({s: bd, s + 2: b}) + embed({s: b, s + 2: bd}))
    return H.tocsr()


def strang_layers(dt: float):
    """Second-order splitting over the three commuting groups j mod 3:
    A(dt/2) B(dt/2) C(dt) B(dt/2) A(dt/2), as (group, tau) pairs in the
    order they act on the state (Appendix A: second-order TEBD)."""
    return [(0, 0.5 * dt), (1, 0.5 * dt), (2, dt), (1, 0.5 * dt), (0, 0.5 * dt)]


def group_sites(L: int, group: int):
    """Left sites j of the gates in group ``group`` (j mod 3 == group)."""
    return list(range(group, L - 2, 3))
