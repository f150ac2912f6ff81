"""Pins of the particle-number bookkeeping (oracle/u1.py) and of the random
U(1) input generator: closed forms on Fock states, the generator's own
sector labels, and the identity sum_a Lambda_a^2 q_b(a) = sum_{i<b} <n_i>
against the independently computed densities."""
import numpy as np
import pytest

from oracle import tebd as otebd
from oracle import u1 as ou1
from workloads import Model, Trunc, cdw_occupations, random_mps_u1, u1_bond_sectors


def test_fock_state_charges_are_prefix_sums():
    occ = [1, 0, 2, 1, 0, 0, 1, 2]
    mps = otebd.MPS.product(3, occ)
    q = ou1.bond_charges(mps)
    pref = np.concatenate([[0], np.cumsum(occ)])
    for b in range(len(occ) + 1):
        assert q[b].shape == (1,)
        assert abs(q[b][0] - pref[b]) < 1e-14


def test_generator_sectors_respect_bounds():
    L, d, chi, N = 10, 3, 12, 5
    mult = u1_bond_sectors(L, d, chi, N)
    assert mult[0] == {0: 1} and mult[L] == {N: 1}
    for b in range(L + 1):
        for q, v in mult[b].items():
            assert v >= 1
            assert 0 <= q <= min(N, b * (d - 1))          # reachable from the left
            assert N - q <= (L - b) * (d - 1)             # and from the right
        assert sum(mult[b].values()) <= min(d ** min(b, L - b), chi)
        if b < L:   # rows of every block of B_b fit in its columns
            for q, v in mult[b].items():
                assert v <= sum(mult[b + 1].get(q + s, 0) for s in range(d))


@pytest.mark.parametrize("L,d,chi,N,seed", [(8, 3, 9, 4, 0), (12, 4, 20, 5, 3), (9, 5, 30, 4, 1)])
def test_generator_blocks_and_charges(L, d, chi, N, seed):
    B, lam, charges = random_mps_u1(L, d, chi, N, seed=seed)
    for i, T in enumerate(B):
        cl, dd, cr = T.shape
        assert (cl, cr) == (len(charges[i]), len(charges[i + 1]))
        # entries outside the sectors q_{i+1} = q_i + s are exactly zero
        allowed = charges[i][:, None, None] + np.arange(d)[None, :, None] == charges[i + 1][None, None, :]
        assert np.all(T[~allowed] == 0)
        Mx = T.reshape(cl, dd * cr)
        assert np.abs(Mx @ Mx.conj().T - np.eye(cl)).max() < 1e-13
    for b in range(L + 1):
        assert abs(np.sum(lam[b] ** 2) - 1.0) < 1e-14
    # the definition recovers the generator's labels exactly
    q = ou1.bond_charges(otebd.MPS([t.copy() for t in B], [l.copy() for l in lam]))
    for b in range(L + 1):
        assert np.abs(q[b] - charges[b]).max() < 1e-12


def test_charges_of_evolved_state_match_densities():
    """After gates the Schmidt vectors keep definite numbers (trap and U break
    degeneracies between sectors), and their Lambda^2-weighted mean is the
    number of bosons left of the bond given by the measured densities."""
    m = Model(L=8, d=3, U=2.7, J=1.0, Jnnn=0.13, K=0.03)
    tr = Trunc(chi_max=12, w_max=1e-12, eps=1e-12)
    res = otebd.run(m, tr, 0.05, 6)
    mps = res["mps"]
    n, _, _ = otebd.measure(mps)
    q = ou1.bond_charges(mps)
    for b in range(1, m.L):
        lam2 = mps.lam[b] ** 2
        assert abs(np.dot(lam2, q[b]) - np.sum(n[:b])) < 1e-10
        # definite numbers where the spectrum is not degenerate across sectors
        s = mps.lam[b]
        gaps = np.abs(np.subtract.outer(s, s)) + np.eye(len(s))
        pure = gaps.min(axis=1) > 1e-6
        assert np.abs(q[b][pure] - np.round(q[b][pure])).max(initial=0.0) < 1e-8


def test_total_number_from_right_recursion():
    """<N> of a CDW is its number of bosons (counting s + 1 bosons for level s
    would add L), and the overlap recursion gives a unit norm."""
    occ = cdw_occupations(6, 1)
    mps = otebd.MPS.product(2, occ)
    R, E = ou1.right_number_matrices(mps)
    assert abs(R[0][0, 0].real - sum(occ)) < 1e-14 and abs(E[0][0, 0] - 1.0) < 1e-14
