"""Particle numbers the library infers from a state's tensors (tebd_opts.u1)
against their definition, on the CPU (tebd_diag_bond_charges is host code).

A bond index carries the number of bosons to its left: the oracle measures it
as the particle number of the left Schmidt vector (oracle/u1.py), and a Fock
product state has the prefix sums of its occupations."""
import numpy as np
import pytest

from oracle import tebd as otebd
from oracle import u1 as ou1
from workloads import random_mps, random_mps_u1


@pytest.fixture(scope="module")
def pt():
    import paper_2401_05301_amd as pt
    return pt


@pytest.mark.parametrize("L,d,chi,N,seed", [(10, 4, 30, 5, 3), (12, 3, 40, 6, 1), (6, 5, 25, 4, 7)])
def test_charges_of_random_u1_states(pt, L, d, chi, N, seed):
    B, lam, labels = random_mps_u1(L, d, chi, N, seed=seed, tau=8.0)
    q = pt.tebd_diag_bond_charges(B)
    oq = ou1.bond_charges(otebd.MPS([b.copy() for b in B], [x.copy() for x in lam]))
    for b in range(L + 1):
        assert np.array_equal(q[b], labels[b]), b
        assert np.abs(oq[b] - q[b]).max() < 1e-8, b
    assert q[0].tolist() == [0] and q[L].tolist() == [N]


def test_charges_of_product_state(pt):
    occ = [1, 0, 2, 1, 0, 3, 1]
    d = 4
    B = []
    for n in occ:
        t = np.zeros((1, d, 1), dtype=np.complex128)
        t[0, n, 0] = 1.0
        B.append(t)
    q = pt.tebd_diag_bond_charges(B)
    assert [int(x[0]) for x in q] == [0] + list(np.cumsum(occ))


def test_state_without_definite_numbers_is_rejected(pt):
    B, lam = random_mps(8, 3, 9, seed=1)
    with pytest.raises(pt.TebdError) as e:
        pt.tebd_diag_bond_charges(B)
    assert e.value.status == pt.TEBD_EINVAL and "definite particle number" in str(e.value)


def test_unreached_index_is_rejected(pt):
    B, lam, _ = random_mps_u1(8, 3, 12, 4, seed=2, tau=8.0)
    B = [b.copy() for b in B]
    B[3][:, :, 0] = 0.0   # index 0 of bond 4 is reached by no entry of its left tensor
    with pytest.raises(pt.TebdError) as e:
        pt.tebd_diag_bond_charges(B)
    assert e.value.status == pt.TEBD_EINVAL and "reached by no" in str(e.value)
