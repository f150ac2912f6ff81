"""Particle-number (U(1)) content of the bonds of an MPS, from its definition.

Test infrastructure: plain FP64 NumPy used to check the GPU library, never
called by it.

Eq. (1) conserves the total boson number, so every Schmidt vector of a state
with N bosons can be chosen with a definite number of bosons on each side of
its bond (Sec. II B keeps the tensors block-sparse in these sectors).  Here
that number is computed from its definition, without assuming any block
structure: for the right-orthonormal B tensors the right Schmidt vectors
|a>_R of bond b span sites b..L-1, and

    q_b(a) = <N> - <a|N_{>=b}|a>_R,     N_{>=b} = sum_{i >= b} n_i,

the bosons left of the bond.  <a|N_{>=b}|a'>_R follows from the recursion
R_b[a, a'] = sum_{s, c, c'} conj(B_b[a, s, c]) B_b[a', s, c'] (s E_{b+1}[c, c'] + R_{b+1}[c, c']),
R_L = 0, with the overlaps E_b[a, a'] = <a|a'>_R from the same recursion
without the number (E_L = 1).  After truncation the stored B are right-
orthonormal only approximately, so each diagonal entry is divided by the
vector's own norm E_b[a, a]; <N> = R_0 / E_0 (bond 0 has one index and no
boson on its left).  For a state with a definite number in every sector
q_b(a) is then an integer.
"""
from __future__ import annotations

from typing import List

import numpy as np

from .tebd import MPS


def right_number_matrices(mps: MPS):
    """(R_b, E_b) for every bond b = 0..L: R_b = <a|N_{>=b}|a'>_R and the
    overlaps E_b = <a|a'>_R (R_L = [[0]], E_L = [[1]])."""
    L = mps.L
    R: List[np.ndarray] = [None] * (L + 1)
    E: List[np.ndarray] = [None] * (L + 1)
    R[L] = np.zeros((1, 1), dtype=np.complex128)
    E[L] = np.ones((1, 1), dtype=np.complex128)
    for b in range(L - 1, -1, -1):
        Bb = mps.B[b]
        d = Bb.shape[1]
        occ = np.arange(d, dtype=np.float64)
        # sum_s s * conj(B[a,s,c]) E[c,c'] B[a',s,c'] + conj(B[a,s,c]) R[c,c'] B[a',s,c']
        local = np.einsum("asc,s,cx,bsx->ab", Bb.conj(), occ, E[b + 1], Bb, optimize=True)
        rest = np.einsum("asc,cx,bsx->ab", Bb.conj(), R[b + 1], Bb, optimize=True)
        R[b] = local + rest
        E[b] = np.einsum("asc,cx,bsx->ab", Bb.conj(), E[b + 1], Bb, optimize=True)
    return R, E


def bond_charges(mps: MPS) -> List[np.ndarray]:
    """q_b(a) for every bond b and index a (real; integers for a state with
    a definite number in every Schmidt sector)."""
    R, E = right_number_matrices(mps)
    N = float((R[0][0, 0] / E[0][0, 0]).real)
    return [N - np.real(np.diag(Rb)) / np.real(np.diag(Eb)) for Rb, Eb in zip(R, E)]
