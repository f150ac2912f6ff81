"""U(1) block-sparse SVDs (tebd_opts.u1) against the dense FP64 oracle.

The sector decomposition reaches the dense result up to rounding order, so
observables, Schmidt spectra (compared after sorting, since the library
orders each bond by particle number), bond dimensions and the ledger are
held to the dense bars, and the particle number the library attaches to
every Schmidt value is checked against its definition (oracle/u1.py)."""
import numpy as np
import pytest

from gpu_util import note
from oracle import supersite as oss
from oracle import tebd as otebd
from oracle import u1 as ou1
from workloads import CONFIGS, Model, Trunc, cdw_occupations, random_mps, random_mps_u1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    import paper_2401_05301_amd as pt
    return pt


def gpu_model(pt, m: Model):
    return pt.make_model(m.L, m.d, m.U, m.J, m.Jnnn, m.K, m.centre())


def bar(om, base=1e-10):
    return base if om.min_gap >= 1e-8 else max(base, 2 * om.w_total)


def check_bonds(g, om, tol, weights=False):
    """Sorted spectra, bond dimensions, the library's order and the particle
    number of every Schmidt value where the oracle's value is isolated.  With
    weights (the Gram route) the squares s^2 are compared to 1e-12: the
    Gram route holds Schmidt weights to about 100 u, a value s ~ 1e-5 to
    ~1e-9, while the observables meet the FP64 bar."""
    assert g.bond_dims() == om.bond_dims()
    q_ref = ou1.bond_charges(om)
    for b in range(1, om.L):
        lam_g, q_g = g.lam(b), g.charges(b)
        assert len(q_g) == len(lam_g)
        assert np.all(np.diff(q_g) >= 0)
        for qq in np.unique(q_g):
            assert np.all(np.diff(lam_g[q_g == qq]) <= 0)
        og = np.argsort(-lam_g, kind="stable")
        oo = np.argsort(-om.lam[b], kind="stable")
        s = om.lam[b][oo]
        if weights:
            assert np.abs(lam_g[og] ** 2 - s ** 2).max() <= 1e-12, b
        else:
            assert np.abs(lam_g[og] - s).max() <= tol, b
        gap = np.full(len(s), np.inf)
        if len(s) > 1:
            dd = np.abs(np.diff(s))
            gap[:-1] = np.minimum(gap[:-1], dd)
            gap[1:] = np.minimum(gap[1:], dd)
        iso = gap > 1e-6
        assert np.all(np.round(q_ref[b][oo][iso]).astype(np.int64) == q_g[og][iso]), b


@pytest.mark.parametrize("svd", [0, 1])
def test_u1_cdw_matches_dense_oracle(pt, svd):
    m = Model(L=10, d=3, U=2.7, J=1.0, Jnnn=0.13, K=0.03)
    # the Gram route takes eps >= 1e-6 (TEBD_GRAM_EPS_MIN); both sides use it
    tr = Trunc(chi_max=16, w_max=1e-12, eps=1e-12 if svd == 0 else 1e-6)
    dt, steps = 0.05, 8
    note(f"u1 cdw L={m.L} d={m.d} chi={tr.chi_max} svd={svd}")
    ores = otebd.run(m, tr, dt, steps)
    g = pt.MPS.cdw(gpu_model(pt, m), pt.make_opts(tr.chi_max, tr.w_max, tr.eps, svd=svd, u1=True))
    tol = bar(ores["mps"])
    for t in range(steps):
        g.step(dt)
        n, C, D = g.measure()
        assert np.abs(n - ores["n"][t]).max() <= tol
        assert np.abs(C - ores["C"][t]).max() <= tol
        assert np.abs(D - ores["D"][t]).max() <= tol
    check_bonds(g, ores["mps"], tol, weights=svd == 1)
    assert abs(g.discarded_weight() - ores["w_total"][-1]) <= 1e-12 + 1e-6 * ores["w_total"][-1]
    g.close()


@pytest.mark.parametrize("svd", [0, 1])
def test_u1_random_state_layers(pt, svd):
    """One layer of each group on a random right-orthonormal state of N = 6
    bosons with many sectors per bond; the library infers the particle
    numbers from the tensors."""
    L, d, chi, N = 12, 4, 40, 6
    B, lam, charges = random_mps_u1(L, d, chi, N, seed=2, tau=8.0)
    m = Model(L=L, d=d, U=3.0, J=1.0, Jnnn=0.1, K=0.01)
    tr = Trunc(chi_max=chi, w_max=1e-12, eps=1e-12 if svd == 0 else 1e-6)
    om = otebd.MPS([b.copy() for b in B], [l.copy() for l in lam])
    g = pt.MPS.from_tensors(gpu_model(pt, m), pt.make_opts(chi, tr.w_max, tr.eps, svd=svd, u1=True), B, lam)
    for b in range(L + 1):
        assert np.array_equal(g.charges(b), charges[b])
    gates = otebd.GateCache(m)
    for group, tau in [(0, 0.03), (1, 0.03), (2, 0.06)]:
        note(f"u1 random layer group={group} svd={svd}")
        otebd.apply_layer(om, gates, group, tau, tr)
        g.layer(group, tau)
        n, C, D = g.measure()
        on, oC, oD = otebd.measure(om)
        tol = bar(om)
        note(f"u1 random layer svd={svd}: max |dn| {np.abs(n - on).max():.3e}")
        assert np.abs(n - on).max() < tol
        assert np.abs(C - oC).max() < tol
        assert np.abs(D - oD).max() < tol
    check_bonds(g, om, bar(om), weights=svd == 1)
    assert abs(g.discarded_weight() - om.w_total) < 1e-12 + 1e-8 * om.w_total
    g.close()


def test_u1_supersite(pt):
    L, d, chi, steps, dt = 12, 3, 20, 6, 0.02
    m = Model(L=L, d=d, U=3.0, J=1.0, Jnnn=0.1, K=0.01)
    tr = Trunc(chi_max=chi, w_max=1e-12, eps=1e-12)
    occ = cdw_occupations(L, 1)
    note(f"u1 super-site L={L} chi={chi}")
    ores = oss.run2(m, tr, dt, steps, occ)
    g = pt.MPS.product(gpu_model(pt, m), pt.make_opts(chi, tr.w_max, tr.eps, supersite=True, u1=True), occ)
    for _ in range(steps):
        g.step(dt)
    n, C, D = g.measure()
    tol = bar(ores["mps"])
    assert np.abs(n - ores["n"][-1]).max() <= tol
    assert np.abs(C - ores["C"][-1]).max() <= tol
    assert np.abs(D - ores["D"][-1]).max() <= tol
    assert g.bond_dims() == ores["mps"].bond_dims()
    # super-site bond K carries the bosons of physical sites 0..2K-1
    pref = np.concatenate([[0], np.cumsum(occ)])
    for K in range(L // 2 + 1):
        w = g.lam(K) ** 2
        assert abs(np.dot(w, g.charges(K)) - np.sum(n[:2 * K])) < 1e-9
    assert g.charges(L // 2)[0] == pref[-1]
    g.close()


def test_u1_config2_shape(pt):
    cfg = CONFIGS["nnn_L32_d5_chi256"]
    m, tr, dt = cfg["model"], cfg["trunc"], cfg["dt"]
    steps = 3
    note("u1 config2 shape")
    ores = otebd.run(m, tr, dt, steps)
    g = pt.MPS.cdw(gpu_model(pt, m), pt.make_opts(tr.chi_max, tr.w_max, tr.eps, u1=True))
    for t in range(steps):
        g.step(dt)
    n, C, D = g.measure()
    tol = bar(ores["mps"])
    assert np.abs(n - ores["n"][-1]).max() <= tol
    assert np.abs(C - ores["C"][-1]).max() <= tol
    assert np.abs(D - ores["D"][-1]).max() <= tol
    check_bonds(g, ores["mps"], tol)
    g.close()


def test_u1_rejects_state_without_definite_numbers(pt):
    L, d, chi = 8, 3, 9
    B, lam = random_mps(L, d, chi, seed=1)
    m = Model(L=L, d=d, U=1.0)
    with pytest.raises(pt.TebdError) as e:
        pt.MPS.from_tensors(gpu_model(pt, m), pt.make_opts(chi, u1=True), B, lam)
    assert e.value.status == pt.TEBD_EINVAL
    g = pt.MPS.cdw(gpu_model(pt, m), pt.make_opts(chi))
    with pytest.raises(pt.TebdError) as e:
        g.charges(0)
    assert e.value.status == pt.TEBD_ESTATE
    g.close()


def test_u1_gram_few_sectors(pt):
    """Gram route on a random state of N = 6 bosons spread over few particle
    numbers per bond (sigma = 1), five layers including the second-order
    pattern, against the oracle with the same singular-value floor."""
    L, d, chi, N = 12, 5, 40, 6
    B, lam, _ = random_mps_u1(L, d, chi, N, seed=5, tau=20.0, sigma=1.0, bias=30.0)
    m = Model(L=L, d=d, U=2.0, J=1.0, Jnnn=0.1, K=0.0)
    # the Gram route takes eps >= 1e-6 (TEBD_GRAM_EPS_MIN); both sides use it
    tr = Trunc(chi_max=chi, w_max=1e-12, eps=1e-6)
    om = otebd.MPS([b.copy() for b in B], [l.copy() for l in lam])
    g = pt.MPS.from_tensors(gpu_model(pt, m), pt.make_opts(chi, tr.w_max, tr.eps, svd=pt.SVD_GRAM_EIG, u1=True), B,
                            lam)
    gates = otebd.GateCache(m)
    for group, tau in [(0, 0.01), (1, 0.01), (2, 0.02), (1, 0.01), (0, 0.01)]:
        note(f"u1 gram subspace layer group={group}")
        otebd.apply_layer(om, gates, group, tau, tr)
        g.layer(group, tau)
        n, C, D = g.measure()
        on, oC, oD = otebd.measure(om)
        tol = bar(om)
        note(f"u1 gram layer group={group}: max |dn| {np.abs(n - on).max():.3e}")
        assert np.abs(n - on).max() < tol, np.abs(n - on).max()
        assert np.abs(C - oC).max() < tol
        assert np.abs(D - oD).max() < tol
    check_bonds(g, om, bar(om), weights=True)
    g.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_u1_fp32_theta_gate(pt, prec):
    """U(1) sectors with the FP32 / split-FP32 theta and gate GEMMs: the
    sectors are found from the particle numbers, not from the values, so the
    FP32 path keeps its 1e-6 bar against the FP64 oracle."""
    m = Model(L=10, d=3, U=2.0, J=1.0, Jnnn=0.1, K=0.01)
    tr = Trunc(chi_max=24, w_max=1e-12, eps=1e-12)
    ores = otebd.run(m, tr, 0.02, 8)
    g = pt.MPS.cdw(gpu_model(pt, m), pt.make_opts(tr.chi_max, tr.w_max, tr.eps, prec=prec, u1=True))
    for _ in range(8):
        g.step(0.02)
    n, C, D = g.measure()
    err = max(np.abs(n - ores["n"][-1]).max(), np.abs(C - ores["C"][-1]).max(), np.abs(D - ores["D"][-1]).max())
    note(f"u1 prec={prec} max observable error {err:.3e}")
    assert err <= 1e-6
    g.close()
