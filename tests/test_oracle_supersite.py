"""The super-site two-site oracle (Sec. II B) against the Hamiltonian of
Eq. (1), brute-force state vectors and the three-site oracle."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import model as mdl
from oracle import supersite as ss
from oracle import tebd
from workloads import Model, Trunc, cdw_occupations

EXACT = Trunc(chi_max=10 ** 6, w_max=0.0, eps=1e-14)


def embed4(G, L, d, first):
    """Dense operator of G acting on physical sites first..first+3 (site 0 slowest)."""
    return np.kron(np.kron(np.eye(d ** first), G), np.eye(d ** (L - first - 4)))


@pytest.mark.parametrize("L,d,Jnnn,K", [(4, 2, 0.3, 0.0), (6, 3, -0.12, 0.01), (8, 2, 0.1, 0.05)])
def test_supersite_split_sums_to_hamiltonian(L, d, Jnnn, K):
    m = Model(L=L, d=d, U=2.5, J=1.0, Jnnn=Jnnn, K=K, jc=(L + 1) / 2 + 0.3)
    H = mdl.full_hamiltonian(m).toarray()
    S = sum(embed4(ss.supersite_term(m, k), L, d, 2 * k) for k in range(L // 2 - 1))
    assert np.abs(S - H).max() < 1e-12


def test_supersite_exact_chi_matches_trotterised_vector():
    L, d, dt, steps = 8, 3, 0.05, 6
    m = Model(L=L, d=d, U=3.0, J=1.0, Jnnn=-0.1, K=0.02)
    occ = cdw_occupations(L, 1)
    res = ss.run2(m, EXACT, dt, steps, occ)
    # brute force: dense gates on the state vector, same layering
    psi = np.zeros(d ** L, dtype=complex)
    psi[int("".join(str(x) for x in occ), d)] = 1.0
    for _ in range(steps):
        for group, tau in ss.supersite_layers(dt):
            for k in range(group, L // 2 - 1, 2):
                psi = embed4(ss.supersite_gate(m, k, tau), L, d, 2 * k) @ psi
    b, num = mdl.boson_ops(d)
    n_ex = []
    for i in range(L):
        op = np.kron(np.kron(np.eye(d ** i), num), np.eye(d ** (L - i - 1)))
        n_ex.append((psi.conj() @ op @ psi).real)
    C_ex = []
    for i in range(L - 1):
        op = np.kron(np.kron(np.eye(d ** i), np.kron(b.T, b)), np.eye(d ** (L - i - 2)))
        C_ex.append(psi.conj() @ op @ psi)
    assert np.abs(res["n"][-1] - np.array(n_ex)).max() < 1e-12
    assert np.abs(res["C"][-1] - np.array(C_ex)).max() < 1e-12
    # D from the dense state too
    D_ex = []
    for i in range(L - 2):
        op = np.kron(np.kron(np.eye(d ** i), np.kron(np.kron(b.T, np.eye(d)), b)), np.eye(d ** (L - i - 3)))
        D_ex.append(psi.conj() @ op @ psi)
    assert np.abs(res["D"][-1] - np.array(D_ex)).max() < 1e-12


def test_supersite_and_three_site_agree_to_trotter_order():
    """Both splittings converge to exp(-iHt): at dt = 0.01 their observables
    agree with the exact evolution (and each other) to O(dt^2)."""
    L, d, dt, steps = 8, 3, 0.01, 40
    m = Model(L=L, d=d, U=5.0, J=1.0, Jnnn=0.1, K=0.005)
    occ = cdw_occupations(L, 1)
    r2 = ss.run2(m, EXACT, dt, steps, occ)
    r3 = tebd.run(m, EXACT, dt, steps)
    from oracle import reference as ref
    ex = ref.exact_evolve(m, ref.cdw_vector(m, 1), dt * steps)
    n_ex = ref.observables(ex, L, d)[0]
    assert np.abs(r2["n"][-1] - n_ex).max() < 1e-4
    assert np.abs(r3["n"][-1] - n_ex).max() < 1e-4
    assert np.abs(r2["n"][-1] - r3["n"][-1]).max() < 1e-4
    assert abs(np.sum(r2["n"][-1]) - L / 2) < 1e-12


def test_supersite_fourth_order_step():
    """Fourth-order super-site steps converge as dt^4 to exp(-iHt)."""
    L, d, t = 6, 3, 0.6
    m = Model(L=L, d=d, U=2.0, J=1.0, Jnnn=0.1, K=0.02)
    occ = cdw_occupations(L, 1)
    from oracle import reference as ref
    ex = ref.exact_evolve(m, ref.cdw_vector(m, 1), t)
    n_ex, C_ex, _ = ref.observables(ex, L, d)
    e = []
    for dt in (0.1, 0.05):
        r = ss.run2(m, EXACT, dt, int(round(t / dt)), occ, order=4)
        e.append(max(np.abs(r["n"][-1] - n_ex).max(), np.abs(r["C"][-1] - C_ex).max()))
    assert e[1] < 1e-7
    assert 13.0 < e[0] / e[1] < 19.0, e[0] / e[1]


def test_supersite_truncation_conserves_norm_and_number():
    L, d = 12, 3
    m = Model(L=L, d=d, U=2.0, J=1.0, Jnnn=0.1, K=0.0)
    res = ss.run2(m, Trunc(chi_max=12, w_max=1e-12, eps=1e-12), 0.02, 30, cdw_occupations(L, 1))
    mps = res["mps"]
    for lam in mps.lam:
        assert abs(np.sum(lam ** 2) - 1.0) < 1e-12
    # the local formulas assume orthonormality, exact only up to the discarded weight
    assert np.abs(np.sum(res["n"], axis=1) - L / 2).max() < L * res["w_total"][-1] + 1e-12
    assert max(mps.bond_dims()) <= 12
    assert res["w_total"][-1] > 0.0
