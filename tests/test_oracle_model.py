"""Pins of oracle.model: operators, the three-site split of Eq. (1), gates."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import model as mdl
from workloads import Model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_boson_ops_algebra():
    for d in (2, 3, 5):
        b, n = mdl.boson_ops(d)
        np.testing.assert_allclose(b.T @ b, n, atol=0)
        comm = b @ b.T - b.T @ b
        # [b, b^+] = 1 except on the truncated top level
        np.testing.assert_allclose(np.diag(comm)[:-1], 1.0, atol=1e-15)
        top = np.zeros(d)
        top[-1] = 1.0
        np.testing.assert_allclose(b.T @ top, 0.0)


def embed(h, j, L, d):
    return np.kron(np.eye(d ** j), np.kron(h, np.eye(d ** (L - j - 3))))


@pytest.mark.parametrize("L,d,U,Jnnn,K,jc", [
    (3, 3, 1.3, 0.2, 0.0, None),
    (5, 3, 2.0, -0.12, 0.01, 3.0),
    (6, 3, 5.0, 0.1, 0.005, 3.5),
    (7, 2, 0.0, 0.0, 0.02, 4.2),
    (4, 5, 3.0, 0.1, 0.03, 2.5),
])
def test_three_site_split_sums_to_hamiltonian(L, d, U, Jnnn, K, jc):
    m = Model(L=L, d=d, U=U, J=1.0, Jnnn=Jnnn, K=K, jc=jc)
    H = mdl.full_hamiltonian(m).toarray()
    S = sum(embed(mdl.three_site_term(m, j), j, L, d) for j in range(L - 2))
    assert np.abs(S - H).max() < 1e-13
    assert np.abs(H - H.T).max() == 0.0


def test_hamiltonian_matrix_elements_from_eq1():
    """Hand-checked entries of Eq. (1) on L=3, d=3: |1,0,1> couplings."""
    m = Model(L=3, d=3, U=2.0, J=1.0, Jnnn=0.3, K=0.4, jc=2.0)
    H = mdl.full_hamiltonian(m).toarray()
    idx = lambda a, b, c: (a * 3 + b) * 3 + c
    # diagonal of |1,0,1>: trap K/2 (x - 2)^2 n at x = 1 and 3 -> 0.2 + 0.2
    assert np.isclose(H[idx(1, 0, 1), idx(1, 0, 1)], 0.4)
    # diagonal of |2,0,0>: U/2 * 2 * 1 + K/2 * 1 * 2 = 2 + 0.4
    assert np.isclose(H[idx(2, 0, 0), idx(2, 0, 0)], 2.4)
    # NN hop |1,0,1> -> |0,1,1>: -J <0,1| b_1^+ b_0 |1,0> = -1
    assert np.isclose(H[idx(0, 1, 1), idx(1, 0, 1)], -1.0)
    # NNN hop |1,0,1> -> |2,0,0>: -Jnnn * sqrt(2) * 1
    assert np.isclose(H[idx(2, 0, 0), idx(1, 0, 1)], -0.3 * np.sqrt(2.0))
    # NN hop into a doubly occupied site |1,0,1> -> |0,0,2>? not NN (distance 2): NNN again
    assert np.isclose(H[idx(0, 0, 2), idx(1, 0, 1)], -0.3 * np.sqrt(2.0))


def test_window_counts():
    L = 9
    assert [mdl.gates_covering_site(L, s) for s in range(L)] == [1, 2, 3, 3, 3, 3, 3, 2, 1]
    assert [mdl.gates_covering_bond(L, s) for s in range(L - 1)] == [1, 2, 2, 2, 2, 2, 2, 1]
    assert [mdl.gates_covering_site(3, s) for s in range(3)] == [1, 1, 1]


def test_gate_is_exponential_and_unitary():
    m = Model(L=6, d=5, U=2.442, J=1.0, Jnnn=-0.12, K=0.01, jc=3.5)
    for j in (0, 2, 3):
        h = mdl.three_site_term(m, j)
        for tau in (0.005, 0.01, 0.0785):
            G = mdl.gate(m, j, tau)
            np.testing.assert_allclose(G, sla.expm(-1j * tau * h), atol=1e-13)
            np.testing.assert_allclose(G.conj().T @ G, np.eye(125), atol=1e-13)
            np.testing.assert_allclose(mdl.gate(m, j, -tau) @ G, np.eye(125), atol=1e-13)


def test_gate_conserves_particle_number():
    m = Model(L=5, d=5, U=3.0, J=1.0, Jnnn=0.1, K=0.01)
    _, num = mdl.boson_ops(5)
    eye = np.eye(5)
    Ntot = mdl.kron3(num, eye, eye) + mdl.kron3(eye, num, eye) + mdl.kron3(eye, eye, num)
    G = mdl.gate(m, 1, 0.3)
    assert np.abs(G @ Ntot - Ntot @ G).max() < 1e-13


def test_strang_schedule():
    layers = mdl.strang_layers(0.01)
    tot = {0: 0.0, 1: 0.0, 2: 0.0}
    for g, tau in layers:
        tot[g] += tau
    assert all(abs(v - 0.01) < 1e-18 for v in tot.values())
    assert layers == layers[::-1]
    assert mdl.group_sites(8, 0) == [0, 3]
    assert mdl.group_sites(8, 1) == [1, 4]
    assert mdl.group_sites(8, 2) == [2, 5]
    # L = 64: 21/21/20 gates -> 104 gate updates per step
    n = sum(len(mdl.group_sites(64, g)) for g, _ in layers)
    assert n == 104


def test_table1_parameters_fixture():
    with open(os.path.join(GOLDEN, "table1_params.json")) as f:
        t = json.load(f)
    assert np.isclose(t["dt"], 0.05 * np.pi / 2)
    for name, p in t["sims"].items():
        assert p["Jnnn"] < 0
        m = Model(L=5, d=3, U=p["U"], J=p["J"], Jnnn=p["Jnnn"], K=p["K"])
        H = mdl.full_hamiltonian(m).toarray()
        S = sum(embed(mdl.three_site_term(m, j), j, 5, 3) for j in range(3))
        assert np.abs(S - H).max() < 1e-13
