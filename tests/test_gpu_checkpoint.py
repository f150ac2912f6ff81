"""Checkpoint and resume (mps_checkpoint / mps_restore).

A restored handle must hold exactly the checkpointed state and ledger (its
own checkpoint image is byte-identical to the one it came from), and
evolving it must continue the original run: the same kernels act on the
same data in one process, so observables, Schmidt values and the ledger
after further steps are held to 1e-12; every case has come out
bit-identical, which the test reports."""
import numpy as np
import pytest

from gpu_util import note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    import paper_2401_05301_amd as pt
    return pt


def snapshot(g):
    n, C, D = g.measure()
    lam = np.concatenate([g.lam(b) for b in range(g.sites + 1)])
    return n, C, D, lam, g.discarded_weight()


CASES = [
    dict(name="dense-jacobi", L=10, d=3, chi=6, kw={}),
    dict(name="dense-gram", L=10, d=3, chi=6, kw=dict(svd=1, eps=1e-6)),
    dict(name="u1", L=10, d=3, chi=6, kw=dict(u1=True)),
    dict(name="supersite", L=8, d=3, chi=9, kw=dict(supersite=True)),
]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_checkpoint_resume_continues_the_run(pt, case, tmp_path):
    note(f"checkpoint {case['name']} L={case['L']} d={case['d']} chi_max={case['chi']}")
    model = pt.make_model(case["L"], case["d"], U=2.0, J=1.0, Jnnn=0.3, K=0.01)
    opts = pt.make_opts(chi_max=case["chi"], w_max=1e-12, **case["kw"])
    dt = 0.1
    a = pt.MPS.cdw(model, opts)
    for _ in range(4):
        a.step(dt)
    assert a.discarded_weight() > 0.0          # truncation is active
    img = a.checkpoint()
    path = str(tmp_path / "state.ptebd")
    a.save(path)
    b = pt.MPS.load(path, model, opts)
    c = pt.MPS.restore(model, opts, img)
    assert np.array_equal(b.checkpoint(), img)
    assert np.array_equal(c.checkpoint(), img)
    assert b.bond_dims() == a.bond_dims()
    if case["kw"].get("u1"):
        for bd in range(a.sites + 1):
            assert np.array_equal(b.charges(bd), a.charges(bd))
    for _ in range(3):
        a.step(dt)
        b.step(dt)
    sa, sb = snapshot(a), snapshot(b)
    assert b.bond_dims() == a.bond_dims()
    bitwise = all(np.array_equal(x, y) for x, y in zip(sa, sb))
    print(f"[gpu] {case['name']}: resumed run bit-identical: {bitwise}", flush=True)
    for x, y in zip(sa[:4], sb[:4]):
        assert np.abs(np.asarray(x) - np.asarray(y)).max() <= 1e-12
    assert abs(sa[4] - sb[4]) <= 1e-12 * max(sa[4], 1e-300) + 1e-300
    for g in (a, b, c):
        g.close()


def test_restore_refuses_a_smaller_bond_cap(pt):
    note("checkpoint into a smaller chi_max")
    model = pt.make_model(10, 3, U=2.0)
    a = pt.MPS.cdw(model, pt.make_opts(chi_max=6))
    for _ in range(4):
        a.step(0.1)
    assert max(a.bond_dims()) == 6
    with pytest.raises(pt.TebdError) as e:
        pt.MPS.restore(model, pt.make_opts(chi_max=4), a.checkpoint())
    assert e.value.status == pt.TEBD_EINVAL
    a.close()
