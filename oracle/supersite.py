"""Super-site two-site TEBD (Sec. II B): the paper's own handling of the NNN
hopping.  Every two physical sites (2K, 2K+1) form one super site of local
dimension D = d^2, which turns the NNN model of Eq. (1) on L sites into a
nearest-neighbour model on L/2 super sites; two-site gates act on
neighbouring super sites (K, K+1), i.e. on physical sites 2K..2K+3.

Test infrastructure: a plain FP64 CPU implementation used to check the GPU
library, never called by it.

Split of Eq. (1) into two-super-site terms (the paper does not spell it
out; the reading here): the NN hop inside a super site and the on-site
terms of its two sites are shared equally by the gates that contain that
super site (one at the chain ends, two in the bulk); the NN hop between
the super sites and both NNN hops across them, (2K, 2K+2) and (2K+1, 2K+3),
belong to gate K alone.  Summed over K this is H exactly.

Layers: second order, A(dt/2) B(dt) A(dt/2) with A = gates K even and
B = gates K odd (each group commutes internally).
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from workloads import Model, Trunc
from . import model as mdl
from .tebd import MPS, _truncate, suzuki4_weights


def _kron(*ops):
    out = ops[0]
    for o in ops[1:]:
        out = np.kron(out, o)
    return out


def gates_containing(Ls: int, K: int) -> int:
    """Two-super-site gates (K', K'+1), 0 <= K' <= Ls-2, containing super site K."""
    return min(K, Ls - 2) - max(0, K - 1) + 1


def supersite_term(m: Model, K: int) -> np.ndarray:
    """h_K on super sites (K, K+1), a d^4 x d^4 Hermitian matrix with index
    order (s_{2K}, s_{2K+1}, s_{2K+2}, s_{2K+3}), s_{2K} slowest."""
    if m.L % 2:
        raise ValueError("the super-site chain needs an even number of physical sites")
    Ls = m.L // 2
    if Ls < 2:
        raise ValueError("two-site gates need at least two super sites")
    d = m.d
    b, _ = mdl.boson_ops(d)
    bd = b.T
    eye = np.eye(d)

    def at(ops: Dict[int, np.ndarray]):
        return _kron(*[ops.get(p, eye) for p in range(4)])

    def hop(p, q, amp):
        return -amp * (at({p: bd, q: b}) + at({p: b, q: bd}))

    h = np.zeros((d ** 4, d ** 4))
    # inside each of the two super sites, shared among the gates containing it
    for side, KK in ((0, K), (1, K + 1)):
        p = 2 * side
        inside = hop(p, p + 1, m.J) + at({p: mdl.onsite_energy(m, 2 * KK)}) + \
            at({p + 1: mdl.onsite_energy(m, 2 * KK + 1)})
        h += inside / gates_containing(Ls, KK)
    # across the two super sites: one NN and two NNN hops
    h += hop(1, 2, m.J)
    h += hop(0, 2, m.Jnnn)
    h += hop(1, 3, m.Jnnn)
    return h


def supersite_gate(m: Model, K: int, tau: float) -> np.ndarray:
    w, v = np.linalg.eigh(supersite_term(m, K))
    return (v * np.exp(-1j * w * tau)) @ v.conj().T


def supersite_layers(dt: float):
    """(group, tau) in the order they act: K even (dt/2), K odd (dt), K even (dt/2)."""
    return [(0, 0.5 * dt), (1, dt), (0, 0.5 * dt)]


def supersite_product(d: int, occ) -> MPS:
    """Fock product state on the super-site chain (index s_{2K} d + s_{2K+1})."""
    if len(occ) % 2:
        raise ValueError("even number of physical sites")
    return MPS.product(d * d, [occ[2 * k] * d + occ[2 * k + 1] for k in range(len(occ) // 2)])


def apply_gate2(mps: MPS, K: int, G: np.ndarray, tr: Trunc) -> None:
    """Two-site gate on super sites K, K+1: one SVD, inverse-free update."""
    D = mps.d
    A, Bm = mps.B[K], mps.B[K + 1]
    cl, cr = A.shape[0], Bm.shape[2]
    psi = np.einsum("asx,xtb->astb", A, Bm, optimize=True).reshape(cl, D * D, cr)
    psip = np.einsum("ps,asb->apb", G, psi, optimize=True)
    theta = mps.lam[K][:, None, None] * psip
    v, s, nrm = _truncate(theta.reshape(cl * D, D * cr), tr, mps)
    k = len(s)
    newA = (psip.reshape(cl * D, D * cr) @ v.conj().T) / nrm
    mps.B[K] = np.ascontiguousarray(newA.reshape(cl, D, k))
    mps.B[K + 1] = np.ascontiguousarray(v.reshape(k, D, cr))
    mps.lam[K + 1] = s


class SupersiteGates:
    def __init__(self, m: Model):
        self.m = m
        self._g: Dict = {}

    def __call__(self, K: int, tau: float) -> np.ndarray:
        key = (K, float(tau))
        if key not in self._g:
            self._g[key] = supersite_gate(self.m, K, tau)
        return self._g[key]


def step2(mps: MPS, gates: SupersiteGates, dt: float, tr: Trunc) -> None:
    Ls = mps.L
    for group, tau in supersite_layers(dt):
        for K in range(group, Ls - 1, 2):
            apply_gate2(mps, K, gates(K, tau), tr)


def step4_2(mps: MPS, gates: SupersiteGates, dt: float, tr: Trunc) -> None:
    """Fourth-order step of the super-site chain: five second-order steps
    with the Suzuki weights of ``oracle.tebd.suzuki4_weights``."""
    for w in suzuki4_weights():
        step2(mps, gates, w * dt, tr)


def measure2(mps: MPS, d: int):
    """Physical n_i, C_i = <b_i^+ b_{i+1}>, D_i = <b_i^+ b_{i+2}> of the
    super-site MPS (right-orthonormal gauge, as the three-site oracle)."""
    Ls, D = mps.L, mps.d
    L = 2 * Ls
    b, num = mdl.boson_ops(d)
    bd = b.T
    eye = np.eye(d)
    # one-site operators on a super site: (operator on the first, on the second physical site)
    first = lambda o: np.kron(o, eye)
    second = lambda o: np.kron(eye, o)
    n = np.zeros(L)
    C = np.zeros(L - 1, dtype=np.complex128)
    Dd = np.zeros(L - 2, dtype=np.complex128)

    def local(K, op):
        w = mps.lam[K] ** 2
        Bk = mps.B[K]
        return np.einsum("a,asb,st,atb->", w, Bk.conj(), op, Bk, optimize=True)

    def two(K, op1, op2):
        w = mps.lam[K] ** 2
        E = np.einsum("a,asy,st,atx->yx", w, mps.B[K].conj(), op1, mps.B[K], optimize=True)
        Bn = mps.B[K + 1]
        return np.einsum("yx,ysc,st,xtc->", E, Bn.conj(), op2, Bn, optimize=True)

    for K in range(Ls):
        n[2 * K] = local(K, first(num)).real
        n[2 * K + 1] = local(K, second(num)).real
        C[2 * K] = local(K, first(bd) @ second(b))
        if K + 1 < Ls:
            C[2 * K + 1] = two(K, second(bd), first(b))
            Dd[2 * K] = two(K, first(bd), first(b))
            if 2 * K + 3 < L:
                Dd[2 * K + 1] = two(K, second(bd), second(b))
    return n, C, Dd


def run2(m: Model, tr: Trunc, dt: float, steps: int, occ, order: int = 2):
    """Evolve the Fock state ``occ`` (even length) and measure after every
    step; ``order`` 4 takes fourth-order steps."""
    if order not in (2, 4):
        raise ValueError("order must be 2 or 4")
    mps = supersite_product(m.d, occ)
    gates = SupersiteGates(m)
    out = {"n": [], "C": [], "D": [], "w_total": []}
    for _ in range(steps):
        (step2 if order == 2 else step4_2)(mps, gates, dt, tr)
        n, C, D = measure2(mps, m.d)
        out["n"].append(n)
        out["C"].append(C)
        out["D"].append(D)
        out["w_total"].append(mps.w_total)
    res = {k: np.array(v) for k, v in out.items()}
    res["mps"] = mps
    return res
