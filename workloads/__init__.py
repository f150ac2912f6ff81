"""Seeded synthetic workloads shared by the CPU oracle and the GPU library.

This module only *produces inputs*: Hamiltonian parameter sets, initial
occupations, random MPS tensors and serving request streams.  It holds none
of the TEBD arithmetic (no gates, no SVDs, no truncation, no measurement), so
that the oracle and the HIP path stay independent of each other while being
fed bit-identical inputs.

Parameter sets follow the quench of Eq. (1) (Sec. I A): on-site interaction U,
nearest-neighbour hopping J (=1, the unit of energy), next-nearest-neighbour
hopping J_NNN and a harmonic trap of strength K centred at j_c, with sites
numbered 1..L in the trap term.  The charge-density-wave start is the Fock
product state of Sec. II B.
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Model:
    """Eq. (1) parameters.  ``jc`` is the trap centre in 1-based site units."""

    L: int
    d: int
    U: float
    J: float = 1.0
    Jnnn: float = 0.0
    K: float = 0.0
    jc: float | None = None

    def centre(self) -> float:
        return (self.L + 1) / 2.0 if self.jc is None else float(self.jc)


@dataclasses.dataclass(frozen=True)
class Trunc:
    """Truncation settings of Sec. II B: bond cap chi_max, discarded-weight
    tolerance w_max and relative singular-value tolerance eps."""

    chi_max: int
    w_max: float = 1e-12
    eps: float = 1e-12


# The five workloads the library is exercised on.  Sizes, couplings and time
# steps are fixed here once; tests shorten horizons, never shapes.
CONFIGS = {
    # L=8 open chain, d=3, exact bond dimension 81, U/J = 5, NN only.
    "exact_L8_d3": dict(model=Model(L=8, d=3, U=5.0, J=1.0, Jnnn=0.0, K=0.0),
                        trunc=Trunc(chi_max=81, w_max=0.0, eps=1e-14),
                        dt=0.01, steps=100),
    # L=32, d=5, NNN hopping and trap centred at 16.5, chi = 256.
    "nnn_L32_d5_chi256": dict(model=Model(L=32, d=5, U=5.0, J=1.0, Jnnn=0.1, K=0.005, jc=16.5),
                              trunc=Trunc(chi_max=256, w_max=1e-12, eps=1e-12),
                              dt=0.01, steps=500),
    # L=64 batched layers, chi grows from 1 to 512, truncation weight 1e-10.
    "batched_L64_chi512": dict(model=Model(L=64, d=5, U=3.0, J=1.0, Jnnn=0.1, K=0.002, jc=32.5),
                               trunc=Trunc(chi_max=512, w_max=1e-10, eps=1e-12),
                               dt=0.01, steps=100),
    # L=64 bulk chi = 1024 throughput workload, U/J = 2, no trap.
    "bulk_L64_chi1024": dict(model=Model(L=64, d=5, U=2.0, J=1.0, Jnnn=0.1, K=0.0, jc=32.5),
                             trunc=Trunc(chi_max=1024, w_max=1e-12, eps=1e-12),
                             dt=0.01, steps=100),
}


def cdw_occupations(L: int, first_occupied: int = 1) -> List[int]:
    """Occupations of the CDW start |1,0,1,0,...> (first_occupied=1) or
    |0,1,0,1,...> (first_occupied=0); 0-based site i."""
    if first_occupied not in (0, 1):
        raise ValueError("first_occupied must be 0 or 1")
    return [1 if (i % 2 == 0) == bool(first_occupied) else 0 for i in range(L)]


def centred_cdw_occupations(L: int, N: int) -> List[int]:
    """Centred charge-density wave with empty wings (Sec. II B): N bosons on
    the sites j = 0, +-2, ..., +-(N-1) counted from the centre site
    (L - 1) / 2, every other site empty.  L and N odd, N <= (L + 1) / 2."""
    if L % 2 == 0 or N % 2 == 0 or N > (L + 1) // 2 or N < 1:
        raise ValueError("L and N must be odd with N <= (L + 1) / 2")
    c = (L - 1) // 2
    occ = [0] * L
    for k in range(-(N - 1), N, 2):
        occ[c + k] = 1
    return occ


def bulk_bond_dims(L: int, d: int, chi: int) -> List[int]:
    """Bond dimensions chi_b = min(d^b, d^(L-b), chi), b = 0..L."""
    out = []
    for b in range(L + 1):
        e = min(b, L - b)
        v = 1
        for _ in range(e):
            v *= d
            if v >= chi:
                v = chi
                break
        out.append(min(v, chi))
    return out


def random_mps(L: int, d: int, chi: int, seed: int = 0, tau: float = 30.0,
               bonds: List[int] | None = None, bias: float | None = None
               ) -> Tuple[List[np.ndarray], List[np.ndarray]]:
    """Random MPS in (B, Lambda) form with right-orthonormal B tensors.

    B_i has shape (chi_i, d, chi_{i+1}); its (chi_i) x (d chi_{i+1}) matrix
    has orthonormal rows (drawn as the conjugate transpose of the Q factor
    of a complex Gaussian).  With ``bias`` the Gaussian's column for right
    bond index b is weighted by exp(-b / bias), so that the row space leans
    on the first right indices and the Schmidt spectra of the state decay
    (roughly as exp(-k / bias)) instead of being flat.  Lambda_b is a decaying
    profile s_k ~ exp(-k / tau) normalised to unit 2-norm; Lambda_0 =
    Lambda_L = [1].  The profile is imposed, not derived, so the state is
    right-canonical but not left-canonical until it is canonicalised.
    """
    rng = np.random.default_rng(seed)
    if bonds is None:
        bonds = bulk_bond_dims(L, d, chi)
    B = []
    for i in range(L):
        cl, cr = bonds[i], bonds[i + 1]
        g = rng.standard_normal((d * cr, cl)) + 1j * rng.standard_normal((d * cr, cl))
        if bias is not None:
            g *= np.tile(np.exp(-np.arange(cr) / bias), d)[:, None]
        q, _ = np.linalg.qr(g)
        B.append(np.ascontiguousarray(q.conj().T.reshape(cl, d, cr)))
    lam = []
    for b in range(L + 1):
        k = np.arange(bonds[b], dtype=np.float64)
        s = np.exp(-k / tau)
        lam.append(s / np.sqrt(np.sum(s * s)))
    return B, lam


def random_mps_device(L: int, d: int, chi: int, seed: int = 0, tau: float = 30.0, bias: float | None = None,
                      device: str = "cuda") -> Tuple[List[np.ndarray], List[np.ndarray]]:
    """The recipe of ``random_mps`` with the Gaussian draws and their QR
    factorisations done by torch on ``device`` (a GPU makes the chi = 1024
    input of L = 64 take seconds instead of minutes).  The random stream is
    torch's generator seeded with ``seed``, so the tensors differ from
    ``random_mps``'s for the same seed, but have the same shapes, the same
    distribution and orthonormal rows.  Returned as host arrays."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    bonds = bulk_bond_dims(L, d, chi)
    B = []
    for i in range(L):
        cl, cr = bonds[i], bonds[i + 1]
        re = torch.randn((d * cr, cl), generator=gen, device=device, dtype=torch.float64)
        im = torch.randn((d * cr, cl), generator=gen, device=device, dtype=torch.float64)
        g = torch.complex(re, im)
        del re, im
        if bias is not None:
            w = torch.exp(-torch.arange(cr, device=device, dtype=torch.float64) / bias).repeat(d)
            g = g * w[:, None]
        q, _ = torch.linalg.qr(g)
        B.append(np.ascontiguousarray(q.conj().T.reshape(cl, d, cr).cpu().numpy()))
        del g, q
    lam = []
    for b in range(L + 1):
        k = np.arange(bonds[b], dtype=np.float64)
        s = np.exp(-k / tau)
        lam.append(s / np.sqrt(np.sum(s * s)))
    return B, lam


def u1_bond_sectors(L: int, d: int, chi: int, N: int, sigma: float = 2.0) -> List[dict]:
    """Particle-number sectors of a random U(1) MPS: for every bond b a dict
    {q: multiplicity}, q the number of bosons left of the bond.

    Bond 0 holds {0: 1} and bond L {N: 1}.  Inner bonds spread
    min(d^b, d^(L-b), chi) indices over the particle numbers q reachable from
    both sides, with weights exp(-(q - N b / L)^2 / (2 sigma^2)), at most as
    many indices per q as there are Fock states of the b sites on the left
    with q bosons and of the L - b sites on the right with N - q, and as the
    bond to the right offers (sum over s of its multiplicity of q + s), so
    that the blocks of a right-orthonormal tensor can have orthonormal rows.
    A last left-to-right pass drops particle numbers the left bond cannot
    reach, so every index is reached from the left.
    """
    targets = bulk_bond_dims(L, d, chi)

    def fock_counts(n_sites):
        c = {0: 1}
        for _ in range(n_sites):
            nxt = {}
            for q, v in c.items():
                for s in range(d):
                    nxt[q + s] = min(chi, nxt.get(q + s, 0) + v)
            c = nxt
        return c

    left = [fock_counts(b) for b in range(L + 1)]
    right = [fock_counts(L - b) for b in range(L + 1)]
    mult: List[dict] = [dict() for _ in range(L + 1)]
    mult[L] = {N: 1}
    mult[0] = {0: 1}
    for b in range(L - 1, 0, -1):
        caps = {}
        for q, lv in left[b].items():
            rv = right[b].get(N - q, 0)
            offer = sum(mult[b + 1].get(q + s, 0) for s in range(d))
            c = min(lv, rv, offer)
            if c > 0:
                caps[q] = c
        qbar = N * b / L
        w = {q: np.exp(-(q - qbar) ** 2 / (2.0 * sigma * sigma)) for q in caps}
        wsum = sum(w.values())
        T = min(targets[b], sum(caps.values()))
        ideal = {q: T * w[q] / wsum for q in caps}
        alloc = {q: min(caps[q], int(round(ideal[q]))) for q in caps}
        while sum(alloc.values()) < T:
            q = max((q for q in caps if alloc[q] < caps[q]), key=lambda q: (ideal[q] - alloc[q], -abs(q - qbar)))
            alloc[q] += 1
        while sum(alloc.values()) > T:
            q = max((q for q in caps if alloc[q] > 0), key=lambda q: (alloc[q] - ideal[q], abs(q - qbar)))
            alloc[q] -= 1
        mult[b] = {q: v for q, v in sorted(alloc.items()) if v > 0}
    for b in range(1, L):
        mult[b] = {q: v for q, v in mult[b].items()
                   if any(mult[b - 1].get(q - s, 0) > 0 for s in range(d))}
    return mult


def random_mps_u1(L: int, d: int, chi: int, N: int, seed: int = 0, tau: float = 30.0,
                  sigma: float = 2.0, bias: float | None = None):
    """Random right-orthonormal MPS with a definite number N of bosons.

    Every bond index carries a particle number q (bosons left of the bond),
    sectors from ``u1_bond_sectors``, indices ordered by q.  B_i[a, s, b] is
    zero unless q_{i+1}[b] = q_i[a] + s; each block of rows with one q_i is
    the conjugate transpose of the Q factor of a complex Gaussian (columns
    for right index rank r inside its sector weighted by exp(-r / bias) when
    ``bias`` is given).  Lambda_b is imposed, not derived: index t of sector q
    gets exp(-(q - N b / L)^2 / (4 sigma^2) - t / tau), normalised.

    Returns (B, lam, charges) with charges[b] the particle numbers of bond b.
    """
    rng = np.random.default_rng(seed)
    mult = u1_bond_sectors(L, d, chi, N, sigma)
    charges = []
    for b in range(L + 1):
        q = []
        for k, v in sorted(mult[b].items()):
            q += [k] * v
        charges.append(np.array(q, dtype=np.int64))
    B = []
    for i in range(L):
        ql, qr = charges[i], charges[i + 1]
        cl, cr = len(ql), len(qr)
        T = np.zeros((cl, d, cr), dtype=np.complex128)
        rank_r = np.zeros(cr, dtype=np.int64)
        for k in np.unique(qr):
            idx = np.nonzero(qr == k)[0]
            rank_r[idx] = np.arange(len(idx))
        for k in np.unique(ql):
            rows = np.nonzero(ql == k)[0]
            cols = [(s, b) for s in range(d) for b in np.nonzero(qr == k + s)[0]]
            if len(cols) < len(rows):
                raise ValueError("sector too small for orthonormal rows")
            g = rng.standard_normal((len(cols), len(rows))) + 1j * rng.standard_normal((len(cols), len(rows)))
            if bias is not None:
                g *= np.array([np.exp(-rank_r[b] / bias) for _, b in cols])[:, None]
            qf, _ = np.linalg.qr(g)
            s_idx = np.array([c[0] for c in cols])
            b_idx = np.array([c[1] for c in cols])
            T[rows[:, None], s_idx[None, :], b_idx[None, :]] = qf.conj().T
        B.append(T)
    lam = []
    for b in range(L + 1):
        q = charges[b]
        t = np.zeros(len(q))
        for k in np.unique(q):
            idx = np.nonzero(q == k)[0]
            t[idx] = np.arange(len(idx))
        v = np.exp(-(q - N * b / L) ** 2 / (4.0 * sigma * sigma) - t / tau)
        lam.append(v / np.sqrt(np.sum(v * v)))
    return B, lam, charges


def serving_requests(n: int = 64, seed: int = 5, rate: float = 1.0, small: bool = False):
    """Poisson stream of quench requests (arrival times in seconds).

    Each request draws L from {16,32,48,64}, chi_max from {128,...,1024}
    (from {16,32,64} when ``small``), U ~ U[2,10], J_NNN = 0.1,
    K ~ U[0, 0.01], horizon ~ U[1, 5] in units of hbar/J and dt = 0.01.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    chis = [16, 32, 64] if small else [128, 256, 512, 1024]
    for r in range(n):
        t += rng.exponential(1.0 / rate)
        L = int(rng.choice([16, 32, 48, 64]))
        out.append(dict(id=r, arrival=t,
                        model=Model(L=L, d=5, U=float(rng.uniform(2.0, 10.0)), J=1.0, Jnnn=0.1,
                                    K=float(rng.uniform(0.0, 0.01))),
                        chi_max=int(rng.choice(chis)),
                        horizon=float(rng.uniform(1.0, 5.0)), dt=0.01))
    return out
