"""Three-site-gate TEBD on an MPS, written step by step in FP64.

Representation (Vidal form, stored inverse-free): B_i = Gamma_i Lambda_{i+1}
with shape (chi_i, d, chi_{i+1}) and Lambda_b, b = 0..L, the Schmidt values
on bond b (the bond left of site b); Lambda_0 = Lambda_L = [1].  The state is
Lambda_0 B_0 B_1 ... B_{L-1}.  B tensors are right-orthonormal, so local
expectation values need only the Lambda on the bond left of the window
(Sec. II B: expectation values computed assuming orthonormality).

Gate update on sites (j, j+1, j+2), with the readings the paper leaves open
fixed as follows:
  * psi = B_j B_{j+1} B_{j+2}, psi' = G psi, theta' = Lambda_j psi'.
  * SVD #1 across bond j+1 of theta' as (chi_l d) x (d^2 chi_r); keep k1
    values (rule in ``truncation_rank``), renormalise them to unit 2-norm
    (Sec. II B) and add the discarded weight to the ledger.
  * SVD #2 across bond j+2 of S1 V1^+ as (k1 d) x (d chi_r); same rule.
  * Inverse-free update: B_j = psi' V1 / |S1|, B_{j+1} = V1^+ V2 / |S2|
    (V1^+ reshaped to (k1 d) x (d chi_r)), B_{j+2} = V2^+,
    Lambda_{j+1} = S1, Lambda_{j+2} = S2 (normalised).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np
import scipy.linalg as sla

from workloads import Model, Trunc, cdw_occupations
from . import model as mdl


@dataclasses.dataclass
class MPS:
    B: List[np.ndarray]
    lam: List[np.ndarray]
    w_total: float = 0.0          # FP64 discarded-weight ledger
    min_gap: float = np.inf       # smallest relative gap at a truncating cut

    @property
    def L(self) -> int:
        return len(self.B)

    @property
    def d(self) -> int:
        return self.B[0].shape[1]

    def bond_dims(self) -> List[int]:
        return [len(x) for x in self.lam]

    def copy(self) -> "MPS":
        return MPS([x.copy() for x in self.B], [x.copy() for x in self.lam], self.w_total, self.min_gap)

    @classmethod
    def product(cls, d: int, occ) -> "MPS":
        """Fock product state: every bond has dimension 1."""
        B = []
        for n in occ:
            if not 0 <= n < d:
                raise ValueError("occupation outside the truncated local space")
            t = np.zeros((1, d, 1), dtype=np.complex128)
            t[0, n, 0] = 1.0
            B.append(t)
        lam = [np.ones(1) for _ in range(len(occ) + 1)]
        return cls(B, lam)

    @classmethod
    def cdw(cls, L: int, d: int, first_occupied: int = 1) -> "MPS":
        """Charge-density-wave start (Sec. II B)."""
        return cls.product(d, cdw_occupations(L, first_occupied))


def truncation_rank(s: np.ndarray, tr: Trunc):
    """Number of singular values kept and the relative discarded weight.

    s is sorted in descending order.  Sec. II B names a bond cap chi_max,
    a discarded-weight tolerance w_max and a relative tolerance eps; they are
    combined as k = max(1, min(chi_max, k_w, k_eps)) where
      k_w   = smallest k whose tail sum_{i>=k} s_i^2 <= w_max * sum_i s_i^2,
      k_eps = number of s_i > eps * s_0.
    Returns (k, tail_k / total).
    """
    s2 = s.astype(np.float64) ** 2
    total = float(np.sum(s2))
    n = len(s2)
    if n == 0 or total == 0.0:
        return 1, 0.0
    # tails[k] = sum_{i >= k} s_i^2, accumulated from the smallest value up
    tails = np.zeros(n + 1)
    acc = 0.0
    for i in range(n - 1, -1, -1):
        acc += s2[i]
        tails[i] = acc
    k_w = n
    for k in range(n + 1):
        if tails[k] <= tr.w_max * total:
            k_w = k
            break
    k_eps = int(np.sum(s > tr.eps * s[0]))
    k = max(1, min(tr.chi_max, k_w, k_eps))
    return k, float(tails[k] / total)


def _svd(M: np.ndarray):
    try:
        return sla.svd(M, full_matrices=False, lapack_driver="gesdd")
    except np.linalg.LinAlgError:
        return sla.svd(M, full_matrices=False, lapack_driver="gesvd")


def _truncate(M: np.ndarray, tr: Trunc, mps: MPS):
    """Truncated SVD of M: returns (V^+ rows kept, normalised S, norm of kept S)."""
    _, s, vh = _svd(M)
    k, w = truncation_rank(s, tr)
    if k < len(s) and s[k] > 0.0:
        mps.min_gap = min(mps.min_gap, float((s[k - 1] - s[k]) / s[0]))
    nrm = float(np.sqrt(np.sum(s[:k] ** 2)))
    mps.w_total += w
    return vh[:k], s[:k] / nrm, nrm


def apply_gate(mps: MPS, j: int, G: np.ndarray, tr: Trunc) -> None:
    """Apply the three-site gate G (d^3 x d^3) to sites j, j+1, j+2 in place."""
    d = mps.d
    A, Bm, C = mps.B[j], mps.B[j + 1], mps.B[j + 2]
    cl, cr = A.shape[0], C.shape[2]
    # psi[a, s1, s2, s3, b] = sum_xy A[a,s1,x] Bm[x,s2,y] C[y,s3,b]
    psi = np.einsum("asx,xty,yub->astub", A, Bm, C, optimize=True).reshape(cl, d ** 3, cr)
    # psi'[a, s', b] = sum_s G[s', s] psi[a, s, b]
    psip = np.einsum("ps,asb->apb", G, psi, optimize=True)
    theta = mps.lam[j][:, None, None] * psip
    # SVD #1 across bond j+1
    v1, s1, n1 = _truncate(theta.reshape(cl * d, d * d * cr), tr, mps)
    k1 = len(s1)
    newA = (psip.reshape(cl * d, d * d * cr) @ v1.conj().T) / n1
    # SVD #2 across bond j+2
    m2 = (s1[:, None] * v1).reshape(k1 * d, d * cr)
    v2, s2, n2 = _truncate(m2, tr, mps)
    k2 = len(s2)
    newB = (v1.reshape(k1 * d, d * cr) @ v2.conj().T) / n2
    mps.B[j] = np.ascontiguousarray(newA.reshape(cl, d, k1))
    mps.B[j + 1] = np.ascontiguousarray(newB.reshape(k1, d, k2))
    mps.B[j + 2] = np.ascontiguousarray(v2.reshape(k2, d, cr))
    mps.lam[j + 1] = s1
    mps.lam[j + 2] = s2


class GateCache:
    """Gates exp(-i h_j tau), built once per (j, tau) for a model."""

    def __init__(self, m: Model):
        self.m = m
        self._g: Dict = {}

    def __call__(self, j: int, tau: float) -> np.ndarray:
        key = (j, float(tau))
        if key not in self._g:
            self._g[key] = mdl.gate(self.m, j, tau)
        return self._g[key]


def apply_layer(mps: MPS, gates: GateCache, group: int, tau: float, tr: Trunc) -> None:
    """All gates of one commuting group; they act on disjoint sites."""
    for j in mdl.group_sites(mps.L, group):
        apply_gate(mps, j, gates(j, tau), tr)


def step(mps: MPS, gates: GateCache, dt: float, tr: Trunc) -> None:
    """One second-order Trotter step (five layers)."""
    for group, tau in mdl.strang_layers(dt):
        apply_layer(mps, gates, group, tau, tr)


def suzuki4_weights() -> List[float]:
    """Time weights of the fourth-order step (Suzuki's symmetric fractal composition).

    The appendix on numerical convergence (time step) checks the
    second-order results against fourth-order pTEBD without naming the
    scheme.  The reading here is Suzuki's symmetric fractal composition
    (Phys. Lett. A 146, 319 (1990)) of five second-order steps,
    S4(dt) = S2(p dt) S2(p dt) S2((1 - 4p) dt) S2(p dt) S2(p dt) with
    p = 1 / (4 - 4^(1/3)): the weights sum to one and their cubes to zero,
    which removes the third-order term of the symmetric S2.
    """
    p = 1.0 / (4.0 - 4.0 ** (1.0 / 3.0))
    return [p, p, 1.0 - 4.0 * p, p, p]


def step4(mps: MPS, gates: GateCache, dt: float, tr: Trunc) -> None:
    """One fourth-order step: five second-order steps of the Suzuki weights."""
    for w in suzuki4_weights():
        step(mps, gates, w * dt, tr)


def measure(mps: MPS):
    """n_i, C_i = <b_i^+ b_{i+1}> and D_i = <b_i^+ b_{i+2}> from local
    contractions in the right-orthonormal gauge (Eqs. (4) and (7)).

    Returns (n[L] real, C[L-1] complex, D[L-2] complex).
    """
    L, d = mps.L, mps.d
    b, _ = mdl.boson_ops(d)
    bd = b.T
    occ = np.arange(d, dtype=np.float64)
    n = np.zeros(L)
    C = np.zeros(max(L - 1, 0), dtype=np.complex128)
    D = np.zeros(max(L - 2, 0), dtype=np.complex128)
    env = []
    for i in range(L):
        w = mps.lam[i] ** 2
        Bi = mps.B[i]
        n[i] = float(np.einsum("a,asb,asb,s->", w, Bi.conj(), Bi, occ).real)
        # left environment carrying b^+ on site i
        env.append(np.einsum("a,asy,st,atx->yx", w, Bi.conj(), bd, Bi, optimize=True))
    for i in range(L - 1):
        Bn = mps.B[i + 1]
        C[i] = np.einsum("yx,ysc,st,xtc->", env[i], Bn.conj(), b, Bn, optimize=True)
    for i in range(L - 2):
        Bn, Bnn = mps.B[i + 1], mps.B[i + 2]
        F = np.einsum("yx,ysc,xsd->cd", env[i], Bn.conj(), Bn, optimize=True)
        D[i] = np.einsum("yx,ysc,st,xtc->", F, Bnn.conj(), b, Bnn, optimize=True)
    return n, C, D


def quasi_local(n: np.ndarray, C: np.ndarray, centre: int):
    """Quasi-local observables of Sec. II B from the local n_j and
    C_j = <b_j^+ b_{j+1}>, with the lattice index j counted from the centre
    site (j = i - centre, so the centre is even):

      N        = sum_j n_j                       (conserved particle number)
      n_odd    = sum_{j odd} n_j / N,  n_even = sum_{j even} n_j / N
      C_even   = sum_{j even} C_j / N            (C_j on the bond j, j+1)
      A e^{i phi} = n_even - n_odd - 2 i Im(C_even)   (tunnel oscillation)
      nu       = (1/N) sum_j (C_j + C_j^*)       (visibility, over every bond)

    Returns a dict with those values (A >= 0, phi in (-pi, pi])."""
    L = len(n)
    j = np.arange(L) - centre
    N = float(np.sum(n))
    n_odd = float(np.sum(n[j % 2 != 0])) / N
    n_even = float(np.sum(n[j % 2 == 0])) / N
    jb = np.arange(L - 1) - centre
    C_even = complex(np.sum(C[jb % 2 == 0])) / N
    z = n_even - n_odd - 2j * C_even.imag
    nu = float(np.sum(C + np.conj(C)).real) / N
    return dict(N=N, n_odd=n_odd, n_even=n_even, C_even=C_even, A=abs(z), phi=float(np.angle(z)), nu=nu)


def to_vector(mps: MPS) -> np.ndarray:
    """Dense state vector Lambda_0 B_0 ... B_{L-1} (small L only); site 0 slowest."""
    psi = mps.lam[0][None, :]                      # (1, chi_0)
    for Bi in mps.B:
        cl, d, cr = Bi.shape
        psi = (psi @ Bi.reshape(cl, d * cr)).reshape(-1, cr)
    return psi[:, 0] * mps.lam[-1][0]


def run(m: Model, tr: Trunc, dt: float, steps: int, first_occupied: int = 1,
        mps: Optional[MPS] = None, callback=None, order: int = 2):
    """Evolve from the CDW (or ``mps``) and measure after every step (Sec. II B);
    ``order`` 4 takes fourth-order steps (``step4``).

    Returns a dict of per-step arrays: n (steps, L), C (steps, L-1),
    D (steps, L-2), w_total (steps,), chi_max (steps,), plus the final MPS.
    """
    if mps is None:
        mps = MPS.cdw(m.L, m.d, first_occupied)
    gates = GateCache(m)
    out = {"n": [], "C": [], "D": [], "w_total": [], "chi": []}
    if order not in (2, 4):
        raise ValueError("order must be 2 or 4")
    for t in range(steps):
        (step if order == 2 else step4)(mps, gates, dt, tr)
        n, C, D = measure(mps)
        out["n"].append(n)
        out["C"].append(C)
        out["D"].append(D)
        out["w_total"].append(mps.w_total)
        out["chi"].append(max(mps.bond_dims()))
        if callback is not None:
            callback(t, mps)
    res = {k: np.array(v) for k, v in out.items()}
    res["mps"] = mps
    return res
