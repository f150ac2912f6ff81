"""Independent references that pin the oracle.

* Dense state vectors (small L): the CDW Fock state evolved either by the
  same three-site gate layers (Trotterized, exact in the MPS limit of no
  truncation) or by exp(-i H t) with H built directly from Eq. (1).
* Non-interacting chains: with U = 0 (or d = 2, where the U term vanishes)
  and NN hopping only, or U = 0 bosons with N <= n_max, every term of Eq. (1)
  is quadratic.  The one-body density matrix of a Fock start then evolves
  under the L x L single-particle propagator P: <b_i^+ b_j>(t) =
  sum_k conj(P_ik) P_jk n_k(0).  P = exp(-i h t) exactly, or the ordered
  product of the 3 x 3 single-particle images of the gates for the
  Trotterized evolution.
* Bulk closed form of the free CDW quench on an infinite NN chain
  (Sec. I B, free model of Cramer et al.): n = 1/2 (1 + J0(4 J t)) on the
  initially occupied sites and 1/2 (1 - J0(4 J t)) on the empty ones.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla
from scipy.special import j0

from workloads import Model, cdw_occupations
from . import model as mdl


# ----------------------------------------------------------------- dense states
def fock_vector(d: int, occ) -> np.ndarray:
    idx = 0
    for n in occ:
        idx = idx * d + n
    v = np.zeros(d ** len(occ), dtype=np.complex128)
    v[idx] = 1.0
    return v


def apply_three_site(psi: np.ndarray, L: int, d: int, j: int, G: np.ndarray) -> np.ndarray:
    """Apply a d^3 x d^3 operator to sites j..j+2 of a dense state."""
    t = psi.reshape(d ** j, d ** 3, d ** (L - j - 3))
    return np.einsum("ps,asb->apb", G, t).reshape(-1)


def trotter_evolve(m: Model, psi: np.ndarray, dt: float, steps: int) -> np.ndarray:
    """Same Strang layers of the same gates, on a dense vector."""
    cache = {}
    for _ in range(steps):
        for group, tau in mdl.strang_layers(dt):
            for j in mdl.group_sites(m.L, group):
                key = (j, tau)
                if key not in cache:
                    cache[key] = mdl.gate(m, j, tau)
                psi = apply_three_site(psi, m.L, m.d, j, cache[key])
    return psi


def exact_evolve(m: Model, psi: np.ndarray, t: float) -> np.ndarray:
    """exp(-i H t) psi with H from Eq. (1) (Krylov action of the sparse H)."""
    H = mdl.full_hamiltonian(m).astype(np.complex128)
    return spla.expm_multiply(-1j * t * H, psi)


def observables(psi: np.ndarray, L: int, d: int):
    """n_i, <b_i^+ b_{i+1}>, <b_i^+ b_{i+2}> of a dense state, normalised by <psi|psi>."""
    b, num = mdl.boson_ops(d)
    bd = b.T
    nrm = np.vdot(psi, psi).real
    t = psi.reshape([d] * L)
    n = np.array([np.vdot(t, _act(t, num, s)).real / nrm for s in range(L)])
    C = np.array([np.vdot(t, _act(_act(t, b, s + 1), bd, s)) / nrm for s in range(L - 1)])
    D = np.array([np.vdot(t, _act(_act(t, b, s + 2), bd, s)) / nrm for s in range(L - 2)])
    return n, C, D


def _act(t: np.ndarray, op: np.ndarray, s: int) -> np.ndarray:
    """Apply a one-site operator to axis s of a dense state tensor."""
    return np.moveaxis(np.tensordot(op, t, axes=([1], [s])), 0, s)


# ----------------------------------------------------------- free particles
def single_particle_h(m: Model) -> np.ndarray:
    """L x L hopping matrix of the quadratic part of Eq. (1) (U dropped)."""
    L = m.L
    h = np.zeros((L, L))
    for i in range(L):
        h[i, i] = 0.5 * m.K * (i + 1 - m.centre()) ** 2
    for i in range(L - 1):
        h[i, i + 1] = h[i + 1, i] = -m.J
    for i in range(L - 2):
        h[i, i + 2] = h[i + 2, i] = -m.Jnnn
    return h


def single_particle_gate_block(m: Model, j: int) -> np.ndarray:
    """3 x 3 single-particle image of h_j (same sharing as the many-body split)."""
    L = m.L
    h = np.zeros((3, 3))
    for p in range(3):
        s = j + p
        h[p, p] = 0.5 * m.K * (s + 1 - m.centre()) ** 2 / mdl.gates_covering_site(L, s)
    h[0, 1] = h[1, 0] = -m.J / mdl.gates_covering_bond(L, j)
    h[1, 2] = h[2, 1] = -m.J / mdl.gates_covering_bond(L, j + 1)
    h[0, 2] = h[2, 0] = -m.Jnnn
    return h


def propagator_exact(m: Model, t: float) -> np.ndarray:
    return sla.expm(-1j * t * single_particle_h(m))


def propagator_trotter(m: Model, dt: float, steps: int) -> np.ndarray:
    """Ordered product of gate images: later gates multiply on the left."""
    L = m.L
    step_u = np.eye(L, dtype=np.complex128)
    for group, tau in mdl.strang_layers(dt):
        for j in mdl.group_sites(L, group):
            g = np.eye(L, dtype=np.complex128)
            g[j:j + 3, j:j + 3] = sla.expm(-1j * tau * single_particle_gate_block(m, j))
            step_u = g @ step_u
    return np.linalg.matrix_power(step_u, steps)


def free_observables(P: np.ndarray, occ):
    """n_i, C_i, D_i from the propagator P and initial occupations."""
    n0 = np.asarray(occ, dtype=np.float64)
    rho = (P.conj() * n0[None, :]) @ P.T        # rho[i, j] = <b_i^+ b_j>
    L = len(occ)
    n = np.real(np.diag(rho)).copy()
    C = np.array([rho[i, i + 1] for i in range(L - 1)])
    D = np.array([rho[i, i + 2] for i in range(L - 2)])
    return n, C, D


def bessel_cdw_density(t, occupied: bool, J: float = 1.0):
    """Bulk density of the free NN CDW quench: 1/2 (1 +- J0(4 J t))."""
    sgn = 1.0 if occupied else -1.0
    return 0.5 * (1.0 + sgn * j0(4.0 * J * np.asarray(t)))


def cdw_vector(m: Model, first_occupied: int = 1) -> np.ndarray:
    return fock_vector(m.d, cdw_occupations(m.L, first_occupied))
