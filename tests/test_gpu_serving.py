"""Serving loop and concurrent stepping: every request gets the result it
would get alone, whatever mix it runs in."""
import numpy as np
import pytest

from gpu_util import note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    import paper_2401_05301_amd as pt
    return pt


def requests(pt):
    rng = np.random.default_rng(21)
    out = []
    for i, (L, chi) in enumerate([(8, 8), (12, 16), (10, 12), (16, 16), (9, 8), (14, 16)]):
        m = pt.make_model(L=L, d=3, U=float(rng.uniform(2, 10)), J=1.0, Jnnn=0.1, K=float(rng.uniform(0, 0.01)))
        out.append(dict(model=m, chi_max=chi, dt=0.01, steps=int(rng.integers(10, 30)), arrival=0.004 * i))
    return out


def alone(pt, r):
    o = pt.make_opts(r["chi_max"], 1e-12, 1e-12, workers=1)
    g = pt.MPS.cdw(r["model"], o)
    g.prepare(r["dt"])
    for _ in range(r["steps"]):
        g.step(r["dt"])
    n, C, D = g.measure()
    w = g.discarded_weight()
    g.close()
    return n, C, D, w


def test_serving_results_match_alone(pt):
    reqs = requests(pt)
    note(f"serving {len(reqs)} requests, 3 slots")
    res = pt.tebd_serve(reqs, max_active=3, hbm_budget=8e9)
    for r, s in zip(reqs, res):
        assert s["status"] == pt.TEBD_OK
        assert s["admitted"] >= s["arrival"] - 1e-9 and s["finished"] >= s["admitted"]
        gates = sum(len(range(g0, r["model"].L - 2, 3)) for g0 in (0, 1, 2, 1, 0))
        assert s["gate_updates"] == r["steps"] * gates
        n, C, D, w = alone(pt, r)
        # identical kernels on identical inputs: equal to rounding (in practice bitwise)
        assert np.abs(s["n"] - n).max() <= 1e-13
        assert np.abs(s["c_nn"] - C).max() <= 1e-13
        assert np.abs(s["c_nnn"] - D).max() <= 1e-13
        assert abs(s["discarded_weight"] - w) <= 1e-15
        assert abs(np.sum(n) - r["model"].L // 2 - r["model"].L % 2) < 1e-9


def test_serving_admits_by_memory(pt):
    reqs = requests(pt)[:4]
    foot = [pt.mps_footprint(r["model"], pt.make_opts(r["chi_max"], workers=1)) for r in reqs]
    note("serving with a budget that fits one request at a time")
    res = pt.tebd_serve(reqs, max_active=4, hbm_budget=float(max(foot)) * 1.01)
    order = sorted(range(len(reqs)), key=lambda i: reqs[i]["arrival"])
    for a, b in zip(order, order[1:]):
        if foot[a] + foot[b] > max(foot) * 1.01:
            assert res[b]["admitted"] >= res[a]["finished"] - 1e-9
    assert all(s["status"] == pt.TEBD_OK for s in res)


def test_step_many_matches_single_steps(pt):
    reqs = requests(pt)[:3]
    note("tebd_step_many on 3 handles vs tebd_step")
    hs, ref = [], []
    for r in reqs:
        o = pt.make_opts(r["chi_max"], 1e-12, 1e-12, workers=1)
        hs.append(pt.MPS.cdw(r["model"], o))
        ref.append(pt.MPS.cdw(r["model"], o))
    for _ in range(12):
        pt.tebd_step_many([g.h for g in hs], [0.01] * len(hs))
        for g in ref:
            g.step(0.01)
    for g, q in zip(hs, ref):
        n1, C1, D1 = g.measure()
        n2, C2, D2 = q.measure()
        assert np.abs(n1 - n2).max() <= 1e-13 and np.abs(C1 - C2).max() <= 1e-13 and np.abs(D1 - D2).max() <= 1e-13
        g.close()
        q.close()


def test_serving_u1_matches_alone_and_dense(pt):
    """Requests served with U(1) sectors give what the same request gives
    alone with U(1) sectors, and agree with the dense route."""
    reqs = requests(pt)[:4]
    note("serving 4 requests with U(1) sectors")
    res = pt.tebd_serve(reqs, max_active=2, hbm_budget=8e9, u1=True)
    for r, s in zip(reqs, res):
        assert s["status"] == pt.TEBD_OK
        o = pt.make_opts(r["chi_max"], 1e-12, 1e-12, workers=1, u1=True)
        g = pt.MPS.cdw(r["model"], o)
        for _ in range(r["steps"]):
            g.step(r["dt"])
        n, C, D = g.measure()
        g.close()
        assert np.abs(s["n"] - n).max() <= 1e-13
        assert np.abs(s["c_nn"] - C).max() <= 1e-13
        nd, Cd, Dd, _ = alone(pt, r)
        # same truncation rule on the same spectra: equal to the dense route
        # within the parity bar (the test chains keep gaps at the cut)
        assert np.abs(n - nd).max() <= 1e-9
        assert np.abs(C - Cd).max() <= 1e-9


def test_fused_step_many_matches_single_steps(pt):
    """tebd_step_many over fused handles (one fused batch per layer across
    all of them, each handle with its own dt) against tebd_step on each."""
    reqs = requests(pt)[:4]
    dts = [0.01, 0.02, 0.015, 0.01]
    note("fused tebd_step_many on 4 handles vs tebd_step")
    hs, ref = [], []
    for r in reqs:
        hs.append(pt.MPS.cdw(r["model"], pt.make_opts(r["chi_max"], 1e-12, 1e-12, fuse=True)))
        ref.append(pt.MPS.cdw(r["model"], pt.make_opts(r["chi_max"], 1e-12, 1e-12, workers=1)))
    for _ in range(15):
        pt.tebd_step_many([g.h for g in hs], dts)
        for g, dt in zip(ref, dts):
            g.step(dt)
    for g, q in zip(hs, ref):
        n1, C1, D1 = g.measure()
        n2, C2, D2 = q.measure()
        assert g.bond_dims() == q.bond_dims()
        assert np.abs(n1 - n2).max() <= 1e-13 and np.abs(C1 - C2).max() <= 1e-13 and np.abs(D1 - D2).max() <= 1e-13
        assert abs(g.discarded_weight() - q.discarded_weight()) <= 1e-15
        for b in range(g.sites + 1):
            assert np.abs(g.lam(b) - q.lam(b)).max() <= 1e-13
        g.close()
        q.close()


def test_batched_serving_matches_alone(pt):
    """Continuous batching: the admitted requests step together, one fused
    batch per layer; every request still gets its result alone."""
    reqs = requests(pt)
    note(f"batched serving of {len(reqs)} requests, 4 slots")
    res = pt.tebd_serve(reqs, max_active=4, hbm_budget=8e9, batched=True, workers_per_request=0, measure_every=5)
    for r, s in zip(reqs, res):
        assert s["status"] == pt.TEBD_OK
        assert s["admitted"] >= s["arrival"] - 1e-9 and s["finished"] >= s["admitted"]
        gates = sum(len(range(g0, r["model"].L - 2, 3)) for g0 in (0, 1, 2, 1, 0))
        assert s["gate_updates"] == r["steps"] * gates
        n, C, D, w = alone(pt, r)
        assert np.abs(s["n"] - n).max() <= 1e-13
        assert np.abs(s["c_nn"] - C).max() <= 1e-13
        assert np.abs(s["c_nnn"] - D).max() <= 1e-13
        assert abs(s["discarded_weight"] - w) <= 1e-15
