"""Pins of the oracle's truncating gate update against its definition on the
dense state vector.

Sec. II B truncates every SVD by discarding the smallest Schmidt values
(bond cap chi_max, weight and relative tolerances) and renormalises the kept
ones.  On a state in canonical (Vidal) form the SVD of theta across a bond
is the Schmidt decomposition of the whole state across that bond, so one
truncating three-site gate update is, by definition:

  psi'  = (1 x G x 1) psi                                  (gate on j..j+2)
  psi1  = top-k1 Schmidt part of psi' across bond j+1, normalised
  psi2  = top-k2 Schmidt part of psi1 across bond j+2, normalised
          (the cut across bond j+1 first, then the one across bond j+2)

Everything below is written here from that definition with numpy's SVD on
the dense vector (L = 6, d = 3, 729 amplitudes), independently of the
oracle's tensor contractions: the canonical input is built from the
Schmidt decompositions of a dense vector, and the oracle's updated MPS must
reproduce psi2 amplitude by amplitude, its new Lambda the kept Schmidt
values, and its ledger the two discarded weights.  A dropped renormalisation,
a Lambda on the wrong side or the mirror SVD order each change psi2 at
O(1) or O(w) and fail these checks (the last test plants two of them).
"""
import numpy as np
import pytest

from oracle import model as mdl
from oracle import tebd as otebd
from workloads import Model, Trunc, random_mps


def contract(B, lam0):
    """Dense vector lam0 B_0 B_1 ... B_{L-1} (site 0 slowest), written out here."""
    v = np.asarray(lam0, dtype=np.complex128).reshape(1, -1)
    for Bi in B:
        cl, d, cr = Bi.shape
        v = (v @ Bi.reshape(cl, d * cr)).reshape(-1, cr)
    return v[:, 0]


def schmidt(psi, L, d, b):
    """Schmidt decomposition of psi across bond b (sites 0..b-1 | b..L-1)."""
    return np.linalg.svd(psi.reshape(d ** b, d ** (L - b)), full_matrices=False)


def canonical_from_vector(psi, L, d, tol=1e-13):
    """Vidal form {B_i = Gamma_i Lambda_{i+1}, Lambda_b} of a normalised dense
    vector: Lambda_b are its Schmidt values across bond b (values below tol
    dropped) and B_i[a, s, c] = <s, R^{(i+1)}_c | R^{(i)}_a> with R^{(b)}_a
    the right Schmidt vectors across bond b (orthonormal rows)."""
    R, lam = [], []
    for b in range(L + 1):
        if b == 0:
            R.append(psi.reshape(1, -1))
            lam.append(np.ones(1))
            continue
        if b == L:
            R.append(np.ones((1, 1), dtype=np.complex128))
            lam.append(np.ones(1))
            continue
        _, s, vh = schmidt(psi, L, d, b)
        k = int(np.sum(s > tol * s[0]))
        R.append(vh[:k])
        lam.append(s[:k])
    B = []
    for i in range(L):
        ra, rc = R[i], R[i + 1]
        t = ra.reshape(ra.shape[0], d, rc.shape[1])
        B.append(np.einsum("asr,cr->asc", t, rc.conj()))
    return B, lam


def apply_three_site(psi, L, d, j, G):
    t = psi.reshape(d ** j, d ** 3, d ** (L - j - 3))
    return np.einsum("ps,asb->apb", G, t).reshape(-1)


def truncate_across(psi, L, d, b, k):
    """Top-k Schmidt part of psi across bond b, renormalised; returns the new
    vector, its normalised kept values and the relative discarded weight."""
    u, s, vh = schmidt(psi, L, d, b)
    kept = s[:k]
    nrm = np.sqrt(np.sum(kept ** 2))
    out = ((u[:, :k] * (kept / nrm)) @ vh[:k]).reshape(-1)
    return out, kept / nrm, float(np.sum(s[k:] ** 2) / np.sum(s ** 2))


def dense_observables(psi, L, d):
    b, _ = mdl.boson_ops(d)   # the textbook truncated annihilator, pinned in test_oracle_model
    occ = np.arange(d, dtype=np.float64)
    t = psi.reshape((d,) * L)
    p = np.abs(t) ** 2
    n = np.array([np.einsum(p, list(range(L)), occ, [i], []) for i in range(L)])

    def on_site(op, site):
        return np.moveaxis(np.tensordot(op, t, axes=([1], [site])), 0, site)

    def corr(i, k):
        # <b+_i b_k> = <b_i psi | b_k psi>
        return complex(np.vdot(on_site(b, i), on_site(b, k)))

    C = np.array([corr(i, i + 1) for i in range(L - 1)])
    D = np.array([corr(i, i + 2) for i in range(L - 2)])
    return n, C, D


def random_state(L, d, seed, chi, tau):
    """A normalised dense vector with decaying Schmidt spectra (from the
    seeded random MPS recipe)."""
    B, lam = random_mps(L, d, chi, seed=seed, tau=tau, bias=4.0)
    psi = contract(B, lam[0])
    return psi / np.linalg.norm(psi)


CASES = [
    # (seed, j, chi_max) with both cuts of the gate active
    (1, 1, 5), (2, 2, 4), (3, 1, 7), (4, 0, 2),
]


@pytest.mark.parametrize("seed,j,chi", CASES)
def test_truncating_gate_update_equals_dense_definition(seed, j, chi):
    L, d = 6, 3
    psi = random_state(L, d, seed, 27, 3.0)
    B, lam = canonical_from_vector(psi, L, d)
    # the constructed Vidal form represents psi
    assert np.abs(contract(B, lam[0]) - psi).max() < 1e-13
    m = Model(L=L, d=d, U=2.5, J=1.0, Jnnn=-0.15, K=0.02)
    G = mdl.gate(m, j, 0.3)
    tr = Trunc(chi_max=chi, w_max=0.0, eps=0.0)
    mps = otebd.MPS([x.copy() for x in B], [x.copy() for x in lam])
    otebd.apply_gate(mps, j, G, tr)
    # the definition on the dense vector
    p1 = apply_three_site(psi, L, d, j, G)
    k1 = min(chi, d ** (j + 1), d ** (L - j - 1))
    p1t, s1, w1 = truncate_across(p1, L, d, j + 1, k1)
    k2 = min(chi, min(d ** (j + 2), d ** (L - j - 2)), k1 * d)
    p2t, s2, w2 = truncate_across(p1t, L, d, j + 2, k2)
    assert w1 > 1e-6 and w2 > 1e-6, (w1, w2)        # both cuts discard weight
    assert mps.bond_dims()[j + 1] == k1 and mps.bond_dims()[j + 2] == k2
    assert np.abs(mps.lam[j + 1] - s1).max() < 1e-12
    assert np.abs(mps.lam[j + 2] - s2).max() < 1e-12
    assert abs(mps.w_total - (w1 + w2)) < 1e-13
    # the updated MPS is the truncated, renormalised state amplitude by amplitude
    v = contract(mps.B, mps.lam[0])
    assert np.abs(v - p2t).max() < 1e-12, np.abs(v - p2t).max()
    # the local measurement (canonical form assumed by its formulas) differs from
    # the exact expectation values of that state by at most O(w)
    n, C, D = otebd.measure(mps)
    ne, Ce, De = dense_observables(p2t, L, d)
    bound = 8.0 * (w1 + w2) * d
    assert np.abs(n - ne).max() <= bound and np.abs(C - Ce).max() <= bound and np.abs(D - De).max() <= bound


def test_untruncated_update_measures_exactly():
    """With every value kept the update is exact and the local measurement
    equals the dense expectation values to rounding."""
    L, d, j = 6, 3, 2
    psi = random_state(L, d, 9, 27, 3.0)
    B, lam = canonical_from_vector(psi, L, d)
    m = Model(L=L, d=d, U=1.5, J=1.0, Jnnn=0.2, K=0.0)
    G = mdl.gate(m, j, 0.2)
    mps = otebd.MPS([x.copy() for x in B], [x.copy() for x in lam])
    otebd.apply_gate(mps, j, G, Trunc(chi_max=10 ** 6, w_max=0.0, eps=1e-14))
    p = apply_three_site(psi, L, d, j, G)
    assert np.abs(contract(mps.B, mps.lam[0]) - p).max() < 1e-12
    n, C, D = otebd.measure(mps)
    ne, Ce, De = dense_observables(p, L, d)
    assert np.abs(n - ne).max() < 1e-12 and np.abs(C - Ce).max() < 1e-12 and np.abs(D - De).max() < 1e-12


def test_pin_catches_planted_mistakes(monkeypatch):
    """Two plausible mistakes planted in the oracle on the CPU: a kept
    spectrum that is not renormalised, and the mirror SVD order.  Both move
    the updated state away from the dense definition by far more than the
    tolerance of the pin above."""
    L, d, j, chi = 6, 3, 1, 5
    psi = random_state(L, d, 1, 27, 3.0)
    B, lam = canonical_from_vector(psi, L, d)
    m = Model(L=L, d=d, U=2.5, J=1.0, Jnnn=-0.15, K=0.02)
    G = mdl.gate(m, j, 0.3)
    tr = Trunc(chi_max=chi, w_max=0.0, eps=0.0)
    p1t, _, _ = truncate_across(apply_three_site(psi, L, d, j, G), L, d, j + 1, chi)
    p2t, _, _ = truncate_across(p1t, L, d, j + 2, chi)
    # mistake 1: the norm of the kept values is not divided out
    real = otebd._truncate

    def no_renorm(M, tr_, mps_):
        vh, s, nrm = real(M, tr_, mps_)
        return vh, s * nrm, 1.0

    monkeypatch.setattr(otebd, "_truncate", no_renorm)
    bad = otebd.MPS([x.copy() for x in B], [x.copy() for x in lam])
    otebd.apply_gate(bad, j, G, tr)
    monkeypatch.setattr(otebd, "_truncate", real)
    assert np.abs(contract(bad.B, bad.lam[0]) - p2t).max() > 1e-4
    # mistake 2: bond j+2 truncated first (the mirror order) gives another state
    q1, _, _ = truncate_across(apply_three_site(psi, L, d, j, G), L, d, j + 2, chi)
    q2, _, _ = truncate_across(q1, L, d, j + 1, chi)
    assert np.abs(q2 - p2t).max() > 1e-4
