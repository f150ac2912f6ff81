"""Fused layers (tebd_opts.fuse): the gates of a layer in lockstep with one
batched one-sided Jacobi per bond.

Each gate goes through the same kernels, launch shapes, tolerances and
sweeps as with concurrent workers, so a fused run must reproduce the
unfused one: observables, every Schmidt spectrum, bond dimensions and the
ledger are compared with the unfused run of the same input, and one case
against the FP64 oracle.  The cases cover both SVD layouts (rows of theta
when chi_l d <= d^2 chi_r, its conjugate transpose with accumulated
vectors near the right edge), more gates than workspaces (the layer is then
fused in chunks), FP32 theta/gate products and a random input with the cap
active from the first layer."""
import time

import numpy as np
import pytest

from gpu_util import note
from oracle import tebd as otebd
from workloads import Model, Trunc, random_mps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    import paper_2401_05301_amd as pt
    return pt


def gpu_model(pt, m: Model):
    return pt.make_model(m.L, m.d, m.U, m.J, m.Jnnn, m.K, m.centre())


def state(g):
    n, C, D = g.measure()
    lam = [g.lam(b) for b in range(g.sites + 1)]
    return n, C, D, lam, g.bond_dims(), g.discarded_weight()


def compare(a, b, what):
    n1, C1, D1, l1, chi1, w1 = a
    n2, C2, D2, l2, chi2, w2 = b
    assert chi1 == chi2, what
    bitwise = (np.array_equal(n1, n2) and np.array_equal(C1, C2) and np.array_equal(D1, D2)
               and all(np.array_equal(x, y) for x, y in zip(l1, l2)) and w1 == w2)
    note(f"{what}: fused bit-identical to unfused: {bitwise}")
    for x, y in ((n1, n2), (C1, C2), (D1, D2)):
        assert np.abs(x - y).max() <= 1e-13, what
    for x, y in zip(l1, l2):
        assert np.abs(x - y).max() <= 1e-13, what
    assert abs(w1 - w2) <= 1e-13 * max(w1, 1e-300) + 1e-300, what


CDW_CASES = [
    dict(name="L11-d3-chi12", L=11, d=3, chi=12, prec=0, workers=0, steps=5),
    dict(name="L11-d3-chi12-two-workspaces", L=11, d=3, chi=12, prec=0, workers=2, steps=5),
    dict(name="L12-d4-chi24-fp32", L=12, d=4, chi=24, prec=1, workers=0, steps=4),
]


@pytest.mark.parametrize("case", CDW_CASES, ids=[c["name"] for c in CDW_CASES])
def test_fused_matches_unfused_from_cdw(pt, case):
    note(f"fused {case['name']}")
    m = Model(L=case["L"], d=case["d"], U=2.0, J=1.0, Jnnn=0.2, K=0.01)
    runs = []
    for fuse in (False, True):
        o = pt.make_opts(case["chi"], 1e-12, 1e-12, prec=case["prec"], workers=case["workers"], fuse=fuse)
        g = pt.MPS.cdw(gpu_model(pt, m), o)
        for _ in range(case["steps"]):
            g.step(0.1)
        runs.append(state(g))
        g.close()
    assert runs[0][5] > 0.0   # the cap truncates
    compare(runs[0], runs[1], case["name"])


def test_fused_random_state_against_oracle(pt):
    """A random right-orthonormal input with the cap active: one layer of
    each group, fused, against the oracle (FP64 bar) and the unfused run."""
    L, d, chi = 10, 4, 16
    B, lam = random_mps(L, d, chi, seed=11, tau=6.0)
    m = Model(L=L, d=d, U=3.0, J=1.0, Jnnn=0.1, K=0.01)
    tr = Trunc(chi_max=chi, w_max=1e-12, eps=1e-12)
    om = otebd.MPS([b.copy() for b in B], [l.copy() for l in lam])
    gates = otebd.GateCache(m)
    runs = []
    for fuse in (False, True):
        g = pt.MPS.from_tensors(gpu_model(pt, m), pt.make_opts(chi, 1e-12, 1e-12, fuse=fuse), B, lam)
        for group, tau in [(0, 0.03), (1, 0.03), (2, 0.06)]:
            g.layer(group, tau)
        runs.append(state(g))
        g.close()
    for group, tau in [(0, 0.03), (1, 0.03), (2, 0.06)]:
        otebd.apply_layer(om, gates, group, tau, tr)
    note("fused random state against the oracle")
    on, oC, oD = otebd.measure(om)
    n, C, D = runs[1][:3]
    tol = 1e-10 if om.min_gap >= 1e-8 else max(1e-10, 2 * om.w_total)
    assert np.abs(n - on).max() < tol
    assert np.abs(C - oC).max() < tol
    assert np.abs(D - oD).max() < tol
    assert runs[1][4] == om.bond_dims()
    assert abs(runs[1][5] - om.w_total) < 1e-12 + 1e-8 * om.w_total
    compare(runs[0], runs[1], "random L10-d4-chi16")


def test_fused_layers_are_faster_at_small_chi(pt):
    """Timing only (reported, not asserted): the L = 64, d = 5 CDW quench at
    chi <= 32, unfused (six workers) against fused (one workspace per gate)."""
    m = Model(L=64, d=5, U=3.0, J=1.0, Jnnn=0.1, K=0.002)
    out = {}
    for fuse in (False, True):
        o = pt.make_opts(32, 1e-10, 1e-10, fuse=fuse)
        g = pt.MPS.cdw(gpu_model(pt, m), o)
        for _ in range(3):
            g.step(0.01)
        g.sync()
        t0 = time.perf_counter()
        for _ in range(20):
            g.step(0.01)
        g.sync()
        out[fuse] = ((time.perf_counter() - t0) / 20, state(g))
        g.close()
    note(f"L=64 d=5 CDW, steps 4-23: unfused {1e3 * out[False][0]:.2f} ms/step, "
         f"fused {1e3 * out[True][0]:.2f} ms/step, max bond {max(out[True][1][4])}")
    compare(out[False][1], out[True][1], "L64-d5 quench")
