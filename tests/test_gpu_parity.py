"""GPU TEBD through the C-ABI against the FP64 CPU oracle, same inputs.

Bars: FP64 path |dn|, |dC|, |dD| <= 1e-10 while every truncating cut has a
relative gap >= 1e-8 (else 2 * w_total + 1e-10); FP32 theta/gate path
<= 1e-6.  Schmidt spectra per bond are compared too (gauge-free)."""
import numpy as np
import pytest

from gpu_util import note
from oracle import tebd as otebd
from workloads import CONFIGS, Model, Trunc, random_mps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    import paper_2401_05301_amd as pt
    return pt


def gpu_model(pt, m: Model):
    return pt.make_model(m.L, m.d, m.U, m.J, m.Jnnn, m.K, m.centre())


def run_pair(pt, m, tr, dt, steps, prec=0, svd=0, first_occupied=1):
    note(f"parity L={m.L} d={m.d} chi={tr.chi_max} steps={steps} prec={prec} svd={svd}")
    ores = otebd.run(m, tr, dt, steps, first_occupied=first_occupied)
    g = pt.MPS.cdw(gpu_model(pt, m), pt.make_opts(tr.chi_max, tr.w_max, tr.eps, prec=prec, svd=svd), first_occupied)
    gn, gc, gd = [], [], []
    for _ in range(steps):
        g.step(dt)
        n, C, D = g.measure()
        gn.append(n); gc.append(C); gd.append(D)
    return ores, g, np.array(gn), np.array(gc), np.array(gd)


GRAM_EPS = 1e-6   # TEBD_GRAM_EPS_MIN: smallest eps the Gram route accepts


def bar(ores, base=1e-10):
    mps = ores["mps"]
    if mps.min_gap < 1e-8:
        return max(base, 2 * ores["w_total"][-1])
    return base


def assert_close(ores, g, gn, gc, gd, tol):
    assert np.abs(gn - ores["n"]).max() <= tol, np.abs(gn - ores["n"]).max()
    assert np.abs(gc - ores["C"]).max() <= tol, np.abs(gc - ores["C"]).max()
    assert np.abs(gd - ores["D"]).max() <= tol, np.abs(gd - ores["D"]).max()


# The Gram route holds Schmidt *weights* s^2 to about 100 u: it takes them
# from a Gram matrix whose eigenvectors near a cut at small s are fixed only
# to u / gap, so a value s ~ 1e-5 can sit 1e-9 away from the oracle's while
# the observables (the FP64 bar) agree to ~1e-11.
GRAM_WEIGHT_TOL = 1e-12


def assert_spectra(ores, g, tol=1e-10, weights=False):
    """Schmidt values per bond against the oracle's, or their squares
    (weights=True, the Gram route) to GRAM_WEIGHT_TOL."""
    assert g.bond_dims() == ores["mps"].bond_dims()
    for b in range(1, g.L):
        ls = g.lam(b)
        lo = ores["mps"].lam[b]
        if weights:
            assert np.abs(ls ** 2 - lo ** 2).max() < GRAM_WEIGHT_TOL, (b, np.abs(ls ** 2 - lo ** 2).max())
        else:
            assert np.abs(ls - lo).max() < tol, (b, np.abs(ls - lo).max())


def test_exact_chi_config1(pt):
    """The exact-chi configuration for its full horizon (100 steps)."""
    cfg = CONFIGS["exact_L8_d3"]
    ores, g, gn, gc, gd = run_pair(pt, cfg["model"], cfg["trunc"], cfg["dt"], cfg["steps"])
    err = max(np.abs(gn - ores["n"]).max(), np.abs(gc - ores["C"]).max(), np.abs(gd - ores["D"]).max())
    note(f"config 1, {cfg['steps']} steps: max observable error {err:.3e}")
    assert_close(ores, g, gn, gc, gd, 1e-10)
    assert_spectra(ores, g, 1e-10)
    assert abs(g.discarded_weight() - ores["w_total"][-1]) < 1e-14


def test_first_occupied_zero_and_nnn_trap(pt):
    m = Model(L=9, d=3, U=2.442, J=1.0, Jnnn=-0.12, K=0.01, jc=5.0)
    tr = Trunc(chi_max=81, w_max=0.0, eps=1e-14)
    ores, g, gn, gc, gd = run_pair(pt, m, tr, 0.05, 10, first_occupied=0)
    assert_close(ores, g, gn, gc, gd, 1e-10)


def test_truncating_nnn_config2_shape(pt):
    cfg = CONFIGS["nnn_L32_d5_chi256"]
    m = cfg["model"]
    tr = Trunc(chi_max=12, w_max=1e-12, eps=1e-12)   # small cap so that truncation is active early
    ores, g, gn, gc, gd = run_pair(pt, m, tr, cfg["dt"], 6)
    assert ores["w_total"][-1] > 0
    assert_close(ores, g, gn, gc, gd, bar(ores))
    assert abs(g.discarded_weight() - ores["w_total"][-1]) < 1e-12 + 1e-6 * ores["w_total"][-1]


def test_config2_full_shape_short(pt):
    cfg = CONFIGS["nnn_L32_d5_chi256"]
    ores, g, gn, gc, gd = run_pair(pt, cfg["model"], cfg["trunc"], cfg["dt"], 3)
    assert_close(ores, g, gn, gc, gd, bar(ores))


def test_gram_variant(pt):
    m = Model(L=8, d=3, U=5.0, J=1.0, Jnnn=0.1, K=0.005)
    # the Gram route takes eps >= 1e-6 (it cannot resolve smaller singular
    # values); both sides apply that eps, and the FP64 bar holds
    tr = Trunc(chi_max=81, w_max=1e-12, eps=GRAM_EPS)
    ores, g, gn, gc, gd = run_pair(pt, m, tr, 0.05, 10, svd=1)
    err = max(np.abs(gn - ores["n"]).max(), np.abs(gc - ores["C"]).max(), np.abs(gd - ores["D"]).max())
    note(f"gram variant L=8: max observable error {err:.3e}, min gap {ores['mps'].min_gap:.2e}")
    assert_close(ores, g, gn, gc, gd, bar(ores))
    assert_spectra(ores, g, weights=True)


def test_gram_route_refuses_eps_below_its_floor(pt):
    m = Model(L=8, d=3, U=5.0, J=1.0)
    with pytest.raises(pt.TebdError) as e:
        pt.MPS.cdw(gpu_model(pt, m), pt.make_opts(16, 1e-12, 1e-12, svd=1))
    assert e.value.status == pt.TEBD_EINVAL
    g = pt.MPS.cdw(gpu_model(pt, m), pt.make_opts(16, 1e-12, 1e-12, svd=0))
    g.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_fp32_theta_gate(pt, prec):
    m = Model(L=10, d=3, U=2.0, J=1.0, Jnnn=0.1, K=0.0)
    tr = Trunc(chi_max=30, w_max=1e-12, eps=1e-12)
    ores, g, gn, gc, gd = run_pair(pt, m, tr, 0.02, 8, prec=prec)
    err = max(np.abs(gn - ores["n"]).max(), np.abs(gc - ores["C"]).max(), np.abs(gd - ores["D"]).max())
    note(f"fp32 prec={prec} max observable error {err:.3e}")
    assert err <= 1e-6


def test_single_layers_and_random_state(pt):
    """One layer of each group on a random right-orthonormal input, chi cap active."""
    L, d, chi = 9, 4, 20
    B, lam = random_mps(L, d, chi, seed=4, tau=6.0)
    m = Model(L=L, d=d, U=3.0, J=1.0, Jnnn=0.1, K=0.01)
    tr = Trunc(chi_max=chi, w_max=1e-12, eps=1e-12)
    om = otebd.MPS([b.copy() for b in B], [l.copy() for l in lam])
    g = pt.MPS.from_tensors(gpu_model(pt, m), pt.make_opts(chi, 1e-12, 1e-12), B, lam)
    n0, C0, D0 = g.measure()
    on, oC, oD = otebd.measure(om)
    assert np.abs(n0 - on).max() < 1e-12 and np.abs(C0 - oC).max() < 1e-12 and np.abs(D0 - oD).max() < 1e-12
    gates = otebd.GateCache(m)
    for group, tau in [(0, 0.03), (1, 0.03), (2, 0.06)]:
        note(f"layer group={group}")
        otebd.apply_layer(om, gates, group, tau, tr)
        g.layer(group, tau)
        n, C, D = g.measure()
        on, oC, oD = otebd.measure(om)
        tol = 1e-10 if om.min_gap >= 1e-8 else max(1e-10, 2 * om.w_total)
        assert np.abs(n - on).max() < tol
        assert np.abs(C - oC).max() < tol
        assert np.abs(D - oD).max() < tol
    assert abs(g.discarded_weight() - om.w_total) < 1e-12 + 1e-8 * om.w_total


@pytest.mark.parametrize("svd", [0, 1])
def test_random_state_layers_chi48(pt, svd):
    """Random right-orthonormal input at chi = 48, d = 5 (Gram matrices of
    at most 240 rows: solved directly on the Gram route)."""
    L, d, chi = 12, 5, 48
    B, lam = random_mps(L, d, chi, seed=7, tau=10.0)
    m = Model(L=L, d=d, U=2.0, J=1.0, Jnnn=0.1, K=0.0)
    tr = Trunc(chi_max=chi, w_max=1e-12, eps=1e-12 if svd == 0 else GRAM_EPS)
    om = otebd.MPS([b.copy() for b in B], [l.copy() for l in lam])
    g = pt.MPS.from_tensors(gpu_model(pt, m), pt.make_opts(chi, tr.w_max, tr.eps, svd=svd), B, lam)
    gates = otebd.GateCache(m)
    errs = []
    for group, tau in [(0, 0.005), (1, 0.005), (2, 0.01)]:
        note(f"chi48 svd={svd} layer group={group}")
        otebd.apply_layer(om, gates, group, tau, tr)
        g.layer(group, tau)
        n, C, D = g.measure()
        on, oC, oD = otebd.measure(om)
        errs.append(max(np.abs(n - on).max(), np.abs(C - oC).max(), np.abs(D - oD).max()))
    note(f"chi48 svd={svd} errors per layer {errs} min_gap {om.min_gap:.2e} w {om.w_total:.2e}")
    tol = 1e-10
    if om.min_gap < 1e-8:
        tol = max(tol, 2 * om.w_total)
    assert max(errs) < tol
    assert g.bond_dims() == om.bond_dims()


def test_layer_workers_give_identical_results(pt):
    """Gates of a layer spread over four concurrent workers give bit-identical
    observables, Schmidt values and ledger to one worker."""
    L, d, chi = 14, 4, 24
    B, lam = random_mps(L, d, chi, seed=3, tau=6.0)
    m = Model(L=L, d=d, U=3.0, J=1.0, Jnnn=0.1, K=0.02)
    res = []
    for workers in (1, 4):
        note(f"workers={workers}")
        g = pt.MPS.from_tensors(gpu_model(pt, m), pt.make_opts(chi, 1e-12, GRAM_EPS, svd=1, workers=workers), B,
                                lam)
        g.step(0.02)
        g.step(0.02)
        n, C, D = g.measure()
        res.append((n, C, D, [g.lam(b) for b in range(L + 1)], g.discarded_weight()))
        g.close()
    a, b = res
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert all(np.array_equal(x, y) for x, y in zip(a[3], b[3]))
    assert a[4] == b[4]


def test_theta_tile_tuner(pt):
    """The theta/gate tile tuner times each new (m, n, k, batch) once per
    handle and reuses its choice; the FP64 result does not depend on the tile
    (both tiles accumulate every element in the same K order), which the
    worker test above also sees, since each handle tunes on its own."""
    L, d, chi = 12, 5, 96
    B, lam = random_mps(L, d, chi, seed=4, tau=20.0)
    m = Model(L=L, d=d, U=2.0, J=1.0, Jnnn=0.1, K=0.0)
    g = pt.MPS.from_tensors(gpu_model(pt, m), pt.make_opts(chi, 1e-12, GRAM_EPS, svd=1, workers=1), B, lam)
    g.layer(2, 0.01)
    t1 = g.tile_tuner()
    g.layer(2, 0.01)
    t2 = g.tile_tuner()
    note(f"tile tuner after one layer {t1}, after two {t2}")
    g.close()
    assert t1["shapes_tuned"] > 0
    assert t2["launches_64"] + t2["launches_128"] > t1["launches_64"] + t1["launches_128"]


@pytest.mark.parametrize("L,N,d,chi,steps", [(41, 11, 3, 24, 6), (121, 27, 5, 16, 3)])
def test_centred_cdw_quasi_local(pt, L, N, d, chi, steps):
    """The experiment's workload shape (Sec. II B): a centred CDW with empty
    wings under simulation [c] of Table I(b), quasi-local observables
    against the oracle's (same state, same truncation)."""
    import json
    import os
    from workloads import centred_cdw_occupations
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_params.json")))
    p = golden["sims"]["c"]
    dt = golden["dt"]
    m = Model(L=L, d=d, U=p["U"], J=p["J"], Jnnn=p["Jnnn"], K=p["K"])
    tr = Trunc(chi_max=chi, w_max=1e-12, eps=1e-12)
    occ = centred_cdw_occupations(L, N)
    centre = (L - 1) // 2
    note(f"centred CDW L={L} N={N} d={d} chi={chi} steps={steps}")
    ores = otebd.run(m, tr, dt, steps, mps=otebd.MPS.product(d, occ))
    g = pt.MPS.product(gpu_model(pt, m), pt.make_opts(chi, tr.w_max, tr.eps), occ)
    for _ in range(steps):
        g.step(dt)
    n, C, D = g.measure()
    tol = bar(ores)
    assert np.abs(n - ores["n"][-1]).max() <= tol
    assert np.abs(C - ores["C"][-1]).max() <= tol
    q = g.quasi_local(centre)
    qo = otebd.quasi_local(ores["n"][-1], ores["C"][-1], centre)
    assert abs(q["N"] - N) < 1e-9
    for key in ("n_odd", "n_even", "A", "phi", "nu"):
        assert abs(q[key] - qo[key]) <= 10 * tol, key
    assert abs(q["C_even"] - qo["C_even"]) <= 10 * tol
    g.close()


@pytest.mark.parametrize("L,d,chi,steps,svd", [(8, 3, 81, 10, 0), (12, 3, 16, 8, 0), (16, 5, 24, 4, 0), (16, 5, 24, 4, 1)])
def test_supersite_two_site_variant(pt, L, d, chi, steps, svd):
    """The paper's super-site chain (Sec. II B, d_eff = d^2, two-site gates)
    against the super-site oracle, same inputs and truncation."""
    from oracle import supersite as oss
    from workloads import cdw_occupations
    m = Model(L=L, d=d, U=3.0, J=1.0, Jnnn=0.1, K=0.01)
    tr = Trunc(chi_max=chi, w_max=0.0 if chi == 81 else 1e-12, eps=1e-14 if chi == 81 else 1e-12)
    if svd == 1:
        tr = Trunc(chi_max=chi, w_max=tr.w_max, eps=GRAM_EPS)
    dt = 0.02
    occ = cdw_occupations(L, 1)
    note(f"super-site L={L} d={d} chi={chi} steps={steps} svd={svd}")
    ores = oss.run2(m, tr, dt, steps, occ)
    g = pt.MPS.product(gpu_model(pt, m), pt.make_opts(chi, tr.w_max, tr.eps, svd=svd, supersite=True), occ)
    assert len(g.bond_dims()) == L // 2 + 1
    for _ in range(steps):
        g.step(dt)
    n, C, D = g.measure()
    tol = bar(ores)
    note(f"super-site svd={svd}: max |dn| {np.abs(n - ores['n'][-1]).max():.3e}")
    assert np.abs(n - ores["n"][-1]).max() <= tol, np.abs(n - ores["n"][-1]).max()
    assert np.abs(C - ores["C"][-1]).max() <= tol, np.abs(C - ores["C"][-1]).max()
    assert np.abs(D - ores["D"][-1]).max() <= tol, np.abs(D - ores["D"][-1]).max()
    assert g.bond_dims() == ores["mps"].bond_dims()
    for b in range(1, L // 2):
        if svd == 0:
            assert np.abs(g.lam(b) - ores["mps"].lam[b]).max() <= tol, b
        else:   # the Gram route resolves weights (see GRAM_WEIGHT_TOL)
            assert np.abs(g.lam(b) ** 2 - ores["mps"].lam[b] ** 2).max() <= GRAM_WEIGHT_TOL, b
    assert abs(g.discarded_weight() - ores["w_total"][-1]) <= 1e-12 + 1e-6 * ores["w_total"][-1]
    g.close()


@pytest.mark.parametrize("svd", [0, 1])
def test_rank_deficient_gram_matrices(pt, svd):
    """A state with definite particle numbers makes every Gram matrix of the
    dense route highly rank-deficient (its rank is the sum of the sector
    ranks).  Identity-gate canonicalisation and two layers against the
    oracle; the Gram route must not lose weight to a subspace stuck in the
    null space (it falls back to the direct solve)."""
    from workloads import random_mps_u1
    L, d, chi = 12, 5, 96
    B, lam, _ = random_mps_u1(L, d, chi, L // 2, seed=0, tau=20.0, bias=30.0)
    m = Model(L=L, d=d, U=2.0, J=1.0, Jnnn=0.1, K=0.0)
    tr = Trunc(chi_max=chi, w_max=1e-12, eps=1e-12 if svd == 0 else GRAM_EPS)
    om = otebd.MPS([b.copy() for b in B], [l.copy() for l in lam])
    eye = np.eye(d ** 3)
    for j in range(L - 2):
        otebd.apply_gate(om, j, eye, tr)
    g = pt.MPS.from_tensors(gpu_model(pt, m), pt.make_opts(chi, tr.w_max, tr.eps, svd=svd), B, lam)
    g.canonicalize()
    note(f"rank-deficient svd={svd}: canonical w {om.w_total:.3e} (GPU {g.discarded_weight():.3e})")
    gates = otebd.GateCache(m)
    for group, tau in [(0, 0.01), (1, 0.01)]:
        otebd.apply_layer(om, gates, group, tau, tr)
        g.layer(group, tau)
    n, C, D = g.measure()
    on, oC, oD = otebd.measure(om)
    tol = bar(ores_like(om))
    note(f"rank-deficient svd={svd}: max |dn| {np.abs(n - on).max():.3e}")
    assert np.abs(n - on).max() < tol, np.abs(n - on).max()
    assert np.abs(C - oC).max() < tol
    assert np.abs(D - oD).max() < tol
    assert abs(g.discarded_weight() - om.w_total) < 1e-10 + 1e-6 * om.w_total
    g.close()


def ores_like(om):
    return {"mps": om, "w_total": [om.w_total]}


@pytest.mark.parametrize("svd", [1, 2])
def test_random_state_layer_gram_subspace_chi256(pt, svd):
    """Gram route where SVD #1 of the central gate has a 1280 x 1280 Gram
    matrix and chi_max = 256: the kept eigenpairs come from the subspace
    iteration, warm-started (svd = 1) or from random rows only (svd = 2, the
    randomised route).  One layer on a random right-orthonormal state,
    against the oracle with the same eps."""
    L, d, chi = 10, 5, 256
    B, lam = random_mps(L, d, chi, seed=3, tau=40.0)
    m = Model(L=L, d=d, U=2.0, J=1.0, Jnnn=0.1, K=0.0)
    tr = Trunc(chi_max=chi, w_max=1e-12, eps=GRAM_EPS)
    om = otebd.MPS([b.copy() for b in B], [l.copy() for l in lam])
    g = pt.MPS.from_tensors(gpu_model(pt, m), pt.make_opts(chi, tr.w_max, tr.eps, svd=svd), B, lam)
    note(f"gram subspace chi=256 layer group=1 svd={svd}")
    otebd.apply_layer(om, otebd.GateCache(m), 1, 0.01, tr)
    g.layer(1, 0.01)
    n, C, D = g.measure()
    on, oC, oD = otebd.measure(om)
    tol = bar(ores_like(om))
    note(f"gram subspace chi=256: max |dn| {np.abs(n - on).max():.3e}, min gap {om.min_gap:.2e}")
    assert np.abs(n - on).max() < tol, np.abs(n - on).max()
    assert np.abs(C - oC).max() < tol
    assert np.abs(D - oD).max() < tol
    assert g.bond_dims() == om.bond_dims()
    assert abs(g.discarded_weight() - om.w_total) < 1e-10 + 1e-6 * om.w_total
    g.close()


def test_fourth_order_step(pt):
    """tebd_step4 (five Strang steps with Suzuki's weights) against
    the oracle's step4 on the exact-chi L=8 chain with NNN hopping and trap,
    and on a truncating chi=20 chain."""
    for m, tr, steps in [
        (Model(L=8, d=3, U=2.0, J=1.0, Jnnn=0.1, K=0.02), Trunc(chi_max=81, w_max=0.0, eps=1e-14), 6),
        (Model(L=10, d=3, U=3.0, J=1.0, Jnnn=-0.1, K=0.01), Trunc(chi_max=20, w_max=1e-12, eps=1e-12), 4),
    ]:
        note(f"fourth order L={m.L} chi={tr.chi_max} steps={steps}")
        ores = otebd.run(m, tr, 0.05, steps, order=4)
        g = pt.MPS.cdw(gpu_model(pt, m), pt.make_opts(tr.chi_max, tr.w_max, tr.eps))
        for _ in range(steps):
            g.step4(0.05)
        n, C, D = g.measure()
        tol = bar(ores)
        assert np.abs(n - ores["n"][-1]).max() <= tol
        assert np.abs(C - ores["C"][-1]).max() <= tol
        assert np.abs(D - ores["D"][-1]).max() <= tol
        if tr.w_max > 0:   # exact chi: the eps cut sits among rounding-level values
            assert g.bond_dims() == ores["mps"].bond_dims()
        g.close()


def test_fourth_order_step_supersite(pt):
    from oracle import supersite as oss
    from workloads import cdw_occupations
    m = Model(L=8, d=2, U=2.0, J=1.0, Jnnn=0.1, K=0.01)
    tr = Trunc(chi_max=16, w_max=0.0, eps=1e-14)
    occ = cdw_occupations(m.L, 1)
    note("fourth order super-site L=8 d=2")
    ores = oss.run2(m, tr, 0.05, 5, occ, order=4)
    g = pt.MPS.product(gpu_model(pt, m), pt.make_opts(tr.chi_max, tr.w_max, tr.eps, supersite=True), occ)
    for _ in range(5):
        g.step4(0.05)
    n, C, D = g.measure()
    tol = bar(ores)
    assert np.abs(n - ores["n"][-1]).max() <= tol
    assert np.abs(C - ores["C"][-1]).max() <= tol
    assert np.abs(D - ores["D"][-1]).max() <= tol
    g.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("svd", [0, 1])
def test_config3_quench_until_truncation_active(pt, svd):
    """The growing-chi quench (L = 64, d = 5, U = 3, J_NNN = 0.1, K = 0.002,
    w_max = 1e-10) from the CDW, compared with the oracle every step until
    well after the truncation has started discarding weight."""
    cfg = CONFIGS["batched_L64_chi512"]
    m, tr, dt = cfg["model"], cfg["trunc"], cfg["dt"]
    if svd == 1:
        tr = Trunc(chi_max=tr.chi_max, w_max=tr.w_max, eps=GRAM_EPS)
    steps = 40
    note(f"config 3 quench svd={svd}: oracle {steps} steps")
    ores = otebd.run(m, tr, dt, steps)
    g = pt.MPS.cdw(gpu_model(pt, m), pt.make_opts(tr.chi_max, tr.w_max, tr.eps, svd=svd))
    errs, first_w = [], None
    for t in range(steps):
        g.step(dt)
        n, C, D = g.measure()
        errs.append(max(np.abs(n - ores["n"][t]).max(), np.abs(C - ores["C"][t]).max(),
                        np.abs(D - ores["D"][t]).max()))
        if first_w is None and ores["w_total"][t] > 0:
            first_w = t
    note(f"config 3 svd={svd}: truncation active from step {first_w}, max bond {max(g.bond_dims())}, "
         f"w {ores['w_total'][-1]:.3e}, max observable error {max(errs):.3e}, min gap {ores['mps'].min_gap:.2e}")
    assert first_w is not None and first_w < steps // 2
    assert max(errs) <= bar(ores)
    assert g.bond_dims() == ores["mps"].bond_dims()
    assert abs(g.discarded_weight() - ores["w_total"][-1]) <= 1e-12 + 1e-6 * ores["w_total"][-1]
    g.close()


@pytest.mark.timeout(900)
def test_config2_chi256_random_input(pt):
    """The NNN + trap chain of configuration 2 (L = 32, d = 5, U = 5,
    J_NNN = 0.1, K = 0.005 centred at 16.5) at chi = 256 from a random
    chi = 256 input: one full Strang step on the Gram route the bench
    times, against the oracle's dense SVDs."""
    cfg = CONFIGS["nnn_L32_d5_chi256"]
    m, dt = cfg["model"], cfg["dt"]
    tr = Trunc(chi_max=256, w_max=cfg["trunc"].w_max, eps=GRAM_EPS)
    B, lam = random_mps(m.L, m.d, 256, seed=11, tau=40.0, bias=60.0)
    om = otebd.MPS([b.copy() for b in B], [l.copy() for l in lam])
    g = pt.MPS.from_tensors(gpu_model(pt, m), pt.make_opts(256, tr.w_max, tr.eps, svd=1), B, lam)
    note("config 2 chi=256: oracle step")
    otebd.step(om, otebd.GateCache(m), dt, tr)
    g.step(dt)
    n, C, D = g.measure()
    on, oC, oD = otebd.measure(om)
    err = max(np.abs(n - on).max(), np.abs(C - oC).max(), np.abs(D - oD).max())
    note(f"config 2 chi=256: max bond {max(g.bond_dims())}, w {om.w_total:.3e}, max observable error {err:.3e}, "
         f"min gap {om.min_gap:.2e}")
    assert max(g.bond_dims()) == 256
    assert err <= bar(ores_like(om))
    assert g.bond_dims() == om.bond_dims()
    assert abs(g.discarded_weight() - om.w_total) <= 1e-12 + 1e-6 * om.w_total
    g.close()
