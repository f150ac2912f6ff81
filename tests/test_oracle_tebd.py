"""Pins of oracle.tebd against brute force, closed forms and invariants."""
import numpy as np
import pytest

from oracle import model as mdl
from oracle import reference as ref
from oracle import tebd
from workloads import CONFIGS, Model, Trunc, cdw_occupations, random_mps

EXACT = Trunc(chi_max=10 ** 6, w_max=0.0, eps=1e-14)


def max_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


# ------------------------------------------------------------ truncation rule
def test_truncation_rank_rules():
    s = np.array([1.0, 0.1, 0.01, 1e-3, 1e-4])
    tot = float(np.sum(s ** 2))
    # chi cap
    assert tebd.truncation_rank(s, Trunc(chi_max=2, w_max=0.0, eps=0.0))[0] == 2
    # weight rule: tail after 3 values is 1e-6 + 1e-8
    k, w = tebd.truncation_rank(s, Trunc(chi_max=10, w_max=1.02e-6 / tot, eps=0.0))
    assert k == 3 and np.isclose(w, (1e-6 + 1e-8) / tot)
    k, _ = tebd.truncation_rank(s, Trunc(chi_max=10, w_max=0.99e-6 / tot, eps=0.0))
    assert k == 4
    # relative rule: strictly greater than eps * s0
    assert tebd.truncation_rank(s, Trunc(chi_max=10, w_max=0.0, eps=1e-3))[0] == 3
    assert tebd.truncation_rank(s, Trunc(chi_max=10, w_max=0.0, eps=0.99e-3))[0] == 4
    # at least one value survives; exact zeros are dropped at w_max = 0
    assert tebd.truncation_rank(s, Trunc(chi_max=10, w_max=1.0, eps=0.0))[0] == 1
    assert tebd.truncation_rank(np.array([1.0, 0.5, 0.0, 0.0]), Trunc(10, 0.0, 0.0))[0] == 2
    assert tebd.truncation_rank(np.array([0.0, 0.0]), Trunc(10, 0.0, 0.0)) == (1, 0.0)


# ------------------------------------------------------ P1: brute force Trotter
@pytest.mark.parametrize("m,steps", [
    (CONFIGS["exact_L8_d3"]["model"], 30),
    (Model(L=7, d=3, U=2.442, J=1.0, Jnnn=-0.12, K=0.01, jc=3.7), 25),
    (Model(L=6, d=4, U=1.0, J=1.0, Jnnn=0.3, K=0.05), 15),
])
def test_exact_chi_matches_trotterized_state_vector(m, steps):
    dt = 0.05
    res = tebd.run(m, EXACT, dt, steps)
    psi = ref.trotter_evolve(m, ref.cdw_vector(m), dt, steps)
    n, C, D = ref.observables(psi, m.L, m.d)
    assert max_err(res["n"][-1], n) < 1e-12
    assert max_err(res["C"][-1], C) < 1e-12
    assert max_err(res["D"][-1], D) < 1e-12
    # the MPS itself equals the Trotterized vector up to a global phase-free identity
    v = tebd.to_vector(res["mps"])
    assert abs(abs(np.vdot(v, psi)) - 1.0) < 1e-12


def test_local_measurement_equals_full_contraction():
    m = Model(L=7, d=3, U=3.0, J=1.0, Jnnn=0.2, K=0.02)
    res = tebd.run(m, EXACT, 0.1, 6)
    mps = res["mps"]
    n, C, D = tebd.measure(mps)
    n2, C2, D2 = ref.observables(tebd.to_vector(mps), m.L, m.d)
    assert max_err(n, n2) < 1e-13 and max_err(C, C2) < 1e-13 and max_err(D, D2) < 1e-13


# ------------------------------------------ P2: exact evolution, O(dt^2) error
def test_trotter_error_is_second_order():
    m = CONFIGS["exact_L8_d3"]["model"]
    t = 1.0
    psi_ex = ref.exact_evolve(m, ref.cdw_vector(m), t)
    n_ex, C_ex, _ = ref.observables(psi_ex, m.L, m.d)
    errs = []
    for dt in (0.02, 0.01):
        res = tebd.run(m, EXACT, dt, int(round(t / dt)))
        errs.append((max_err(res["n"][-1], n_ex), max_err(res["C"][-1], C_ex)))
    assert errs[1][0] < 1e-5 and errs[1][1] < 1e-5
    ratio_n = errs[0][0] / errs[1][0]
    assert 3.5 < ratio_n < 4.5, ratio_n


def test_trotter_error_with_nnn_and_trap():
    m = Model(L=6, d=3, U=2.0, J=1.0, Jnnn=-0.12, K=0.05, jc=3.5)
    t = 0.6
    psi_ex = ref.exact_evolve(m, ref.cdw_vector(m), t)
    n_ex, C_ex, D_ex = ref.observables(psi_ex, m.L, m.d)
    e = []
    for dt in (0.04, 0.02):
        res = tebd.run(m, EXACT, dt, int(round(t / dt)))
        e.append(max(max_err(res["n"][-1], n_ex), max_err(res["C"][-1], C_ex),
                     max_err(res["D"][-1], D_ex)))
    assert e[1] < 1e-4
    assert 3.3 < e[0] / e[1] < 4.7


def test_suzuki_weights_closed_form():
    """The fourth-order weights sum to one and their cubes to zero (the
    condition that removes the third-order term of a symmetric step)."""
    w = tebd.suzuki4_weights()
    assert len(w) == 5 and w == w[::-1]
    assert abs(sum(w) - 1.0) < 1e-15
    assert abs(sum(x ** 3 for x in w)) < 1e-15
    assert w[2] < 0 < w[0]


def test_trotter_error_is_fourth_order():
    """Fourth-order steps against exp(-iHt): halving dt divides the error by
    about 16 (a wrong weight would leave the second-order factor 4)."""
    m = Model(L=6, d=3, U=2.0, J=1.0, Jnnn=-0.12, K=0.05, jc=3.5)
    t = 0.6
    psi_ex = ref.exact_evolve(m, ref.cdw_vector(m), t)
    n_ex, C_ex, D_ex = ref.observables(psi_ex, m.L, m.d)
    e = []
    for dt in (0.1, 0.05):
        res = tebd.run(m, EXACT, dt, int(round(t / dt)), order=4)
        e.append(max(max_err(res["n"][-1], n_ex), max_err(res["C"][-1], C_ex),
                     max_err(res["D"][-1], D_ex)))
    assert e[1] < 1e-7
    assert 13.0 < e[0] / e[1] < 19.0, e[0] / e[1]
    # the second-order step at the same dt is orders of magnitude worse
    r2 = tebd.run(m, EXACT, 0.05, int(round(t / 0.05)))
    assert max_err(r2["n"][-1], n_ex) > 100 * e[1]


# --------------------------------------------------- P3: free fermions (d = 2)
def test_hard_core_matches_free_fermion_propagator():
    m = Model(L=12, d=2, U=7.0, J=1.0, Jnnn=0.0, K=0.005)
    dt, steps = 0.05, 30
    occ = cdw_occupations(m.L, 1)
    res = tebd.run(m, EXACT, dt, steps)
    n, C, _ = ref.free_observables(ref.propagator_trotter(m, dt, steps), occ)
    assert max_err(res["n"][-1], n) < 1e-12
    assert max_err(res["C"][-1], C) < 1e-12


def test_free_propagator_bulk_bessel_closed_form():
    m = Model(L=64, d=2, U=0.0, J=1.0, Jnnn=0.0, K=0.0)
    occ = cdw_occupations(m.L, 1)
    for t in (0.25, 1.0, 2.5, 5.0):
        n, _, _ = ref.free_observables(ref.propagator_exact(m, t), occ)
        for i in (31, 32):
            exp = ref.bessel_cdw_density(t, occupied=bool(occ[i]))
            assert abs(n[i] - exp) < 1e-12, (t, i, n[i], exp)


def test_hard_core_tebd_bulk_bessel():
    """TEBD of a long hard-core chain against 1/2(1 +- J0(4t)) in the bulk."""
    m = Model(L=24, d=2, U=0.0, J=1.0, Jnnn=0.0, K=0.0)
    dt, steps = 0.01, 60
    res = tebd.run(m, Trunc(chi_max=64, w_max=1e-14, eps=1e-12), dt, steps)
    occ = cdw_occupations(m.L, 1)
    n_ex, _, _ = ref.free_observables(ref.propagator_exact(m, dt * steps), occ)
    for i in (11, 12):
        assert abs(res["n"][-1][i] - ref.bessel_cdw_density(dt * steps, bool(occ[i]))) < 1e-5
        assert abs(res["n"][-1][i] - n_ex[i]) < 1e-5


# --------------------------------- P4: free soft-core bosons with N <= n_max
@pytest.mark.parametrize("Jnnn,K", [(0.1, 0.01), (-0.12, 0.0), (0.0, 0.03)])
def test_free_bosons_match_propagator(Jnnn, K):
    m = Model(L=8, d=5, U=0.0, J=1.0, Jnnn=Jnnn, K=K)
    dt, steps = 0.05, 12
    occ = cdw_occupations(m.L, 1)      # N = 4 = n_max
    res = tebd.run(m, EXACT, dt, steps)
    n, C, D = ref.free_observables(ref.propagator_trotter(m, dt, steps), occ)
    assert max_err(res["n"][-1], n) < 1e-11
    assert max_err(res["C"][-1], C) < 1e-11
    assert max_err(res["D"][-1], D) < 1e-11


def test_free_propagator_against_many_body_exact():
    m = Model(L=6, d=4, U=0.0, J=1.0, Jnnn=0.2, K=0.04)
    occ = cdw_occupations(m.L, 0)
    psi = ref.exact_evolve(m, ref.fock_vector(m.d, occ), 0.9)
    n, C, D = ref.observables(psi, m.L, m.d)
    n2, C2, D2 = ref.free_observables(ref.propagator_exact(m, 0.9), occ)
    assert max_err(n, n2) < 1e-12 and max_err(C, C2) < 1e-12 and max_err(D, D2) < 1e-12


# ----------------------------------------------------------- P5: conservation
def test_conservation_under_truncation():
    m = Model(L=10, d=4, U=2.0, J=1.0, Jnnn=0.1, K=0.01)
    tr = Trunc(chi_max=6, w_max=1e-12, eps=1e-12)
    res = tebd.run(m, tr, 0.05, 20)
    N = sum(cdw_occupations(m.L, 1))
    assert res["w_total"][-1] > 1e-8          # it did truncate
    mps = res["mps"]
    for lam in mps.lam:
        assert abs(np.sum(lam ** 2) - 1.0) < 1e-14
    # particle number is conserved by every gate and every truncation of a
    # number-conserving state up to the discarded weight
    assert abs(np.sum(res["n"][-1]) - N) < 10 * N * res["w_total"][-1] + 1e-12
    assert max(mps.bond_dims()) <= 6


def test_exact_norm_and_number():
    m = CONFIGS["exact_L8_d3"]["model"]
    res = tebd.run(m, EXACT, 0.05, 10)
    v = tebd.to_vector(res["mps"])
    assert abs(np.vdot(v, v).real - 1.0) < 1e-13
    assert abs(np.sum(res["n"][-1]) - 4.0) < 1e-12


# ---------------------------------------------------------- P6: time reversal
def test_time_reversal():
    m = Model(L=8, d=3, U=5.0, J=1.0, Jnnn=0.1, K=0.005, jc=4.5)
    mps = tebd.MPS.cdw(m.L, m.d, 1)
    g = tebd.GateCache(m)
    for _ in range(8):
        tebd.step(mps, g, 0.05, EXACT)
    for _ in range(8):
        tebd.step(mps, g, -0.05, EXACT)
    n, C, D = tebd.measure(mps)
    assert max_err(n, cdw_occupations(m.L, 1)) < 1e-12
    assert np.abs(C).max() < 1e-12 and np.abs(D).max() < 1e-12


# ---------------------------------------------------------- P7: special cases
def test_no_hopping_freezes_densities():
    m = Model(L=9, d=5, U=4.0, J=0.0, Jnnn=0.0, K=0.02)
    res = tebd.run(m, EXACT, 0.1, 10, first_occupied=0)
    assert max_err(res["n"][-1], cdw_occupations(9, 0)) < 1e-14
    assert max(res["mps"].bond_dims()) == 1


def test_first_occupied_parity_mirror():
    """Reflection x -> L+1-x maps the even-L CDW |1,0,..> onto |..,0,1>."""
    m = Model(L=8, d=3, U=3.0, J=1.0, Jnnn=0.2, K=0.01, jc=4.5)
    a = tebd.run(m, EXACT, 0.05, 6, first_occupied=1)
    b = tebd.run(m, EXACT, 0.05, 6, first_occupied=0)
    # Strang layers are not reflection symmetric, so compare to O(dt^2)
    assert max_err(a["n"][-1], b["n"][-1][::-1]) < 1e-3


def test_random_mps_input_is_right_orthonormal():
    B, lam = random_mps(8, 5, 16, seed=1)
    for Bi in B:
        cl, d, cr = Bi.shape
        M = Bi.reshape(cl, d * cr)
        np.testing.assert_allclose(M @ M.conj().T, np.eye(cl), atol=1e-13)
    for l in lam:
        assert abs(np.sum(l ** 2) - 1.0) < 1e-14


def test_gate_update_on_random_mps_keeps_gauge():
    """After one truncated gate the new B tensors are right-orthonormal and
    the two new Schmidt vectors are normalised."""
    B, lam = random_mps(6, 5, 40, seed=2, tau=8.0)
    mps = tebd.MPS(B, lam)
    m = Model(L=6, d=5, U=2.0, J=1.0, Jnnn=0.1, K=0.0)
    tr = Trunc(chi_max=40, w_max=1e-12, eps=1e-12)
    tebd.apply_gate(mps, 2, mdl.gate(m, 2, 0.01), tr)
    for i in (3, 4):
        Bi = mps.B[i]
        cl, d, cr = Bi.shape
        M = Bi.reshape(cl, d * cr)
        np.testing.assert_allclose(M @ M.conj().T, np.eye(cl), atol=1e-12)
    for b in (3, 4):
        assert abs(np.sum(mps.lam[b] ** 2) - 1.0) < 1e-14
    assert mps.w_total > 0


# ---------------------------------------------------------------- quasi-local observables (Sec. II B)
def test_centred_cdw_occupations():
    from workloads import centred_cdw_occupations
    occ = centred_cdw_occupations(121, 27)
    assert sum(occ) == 27 and len(occ) == 121
    c = 60
    # the centre (j = 0) is occupied, odd j are empty, wings of equal length
    assert occ[c] == 1 and all(occ[c + j] == 0 for j in range(-59, 60, 2))
    first = occ.index(1)
    last = len(occ) - 1 - occ[::-1].index(1)
    assert c - first == last - c == 26


def test_quasi_local_initial_state_and_hand_example():
    quasi_local = tebd.quasi_local
    from workloads import centred_cdw_occupations
    occ = np.array(centred_cdw_occupations(21, 5), dtype=float)
    q = quasi_local(occ, np.zeros(20, dtype=complex), 10)
    # CDW on the even sites: n_even = 1, n_odd = 0, A = 1, phi = 0, nu = 0
    assert q["N"] == 5 and q["n_odd"] == 0.0 and q["n_even"] == 1.0
    assert q["A"] == 1.0 and q["phi"] == 0.0 and q["nu"] == 0.0
    # hand example: L = 5, centre 2 (j = -2..2), bonds j = -2..1
    n = np.array([0.1, 0.2, 0.3, 0.4, 0.5])
    C = np.array([0.1 + 0.2j, 0.3 - 0.1j, -0.2 + 0.05j, 0.05 + 0.0j])
    q = quasi_local(n, C, 2)
    N = 1.5
    assert np.isclose(q["n_even"], (0.1 + 0.3 + 0.5) / N) and np.isclose(q["n_odd"], (0.2 + 0.4) / N)
    ce = (C[0] + C[2]) / N          # bonds j = -2 and j = 0
    assert np.isclose(q["C_even"], ce)
    z = q["n_even"] - q["n_odd"] - 2j * ce.imag
    assert np.isclose(q["A"], abs(z)) and np.isclose(q["phi"], np.angle(z))
    assert np.isclose(q["nu"], 2 * np.sum(C.real) / N)


def test_quasi_local_free_fermion_centred_cdw():
    """Hard-core bosons (d = 2) from a centred CDW with empty wings: the
    quasi-local values of the oracle's TEBD equal those of the Trotterised
    free-fermion propagator (same dt, no truncation)."""
    from workloads import centred_cdw_occupations
    L, N, dt, steps = 13, 5, 0.05, 20
    occ = centred_cdw_occupations(L, N)
    m = Model(L=L, d=2, U=0.0, J=1.0, Jnnn=0.0, K=0.0)
    mps = tebd.MPS.product(2, occ)
    gates = tebd.GateCache(m)
    for _ in range(steps):
        tebd.step(mps, gates, dt, Trunc(chi_max=64, w_max=0.0, eps=1e-14))
    n, C, _ = tebd.measure(mps)
    q = tebd.quasi_local(n, C, (L - 1) // 2)
    n_ex, C_ex, _ = ref.free_observables(ref.propagator_trotter(m, dt, steps), occ)
    q_ex = tebd.quasi_local(n_ex, C_ex, (L - 1) // 2)
    assert abs(q["N"] - N) < 1e-12
    for key in ("n_odd", "n_even", "A", "phi", "nu"):
        assert abs(q[key] - q_ex[key]) < 1e-10, key
    assert abs(q["C_even"] - q_ex["C_even"]) < 1e-10
    # the wave has begun to relax: particles have moved onto the odd sites
    assert 0.05 < q["n_odd"] < 0.95
