"""Full-size checks in the configuration bench.py times (d = 5, chi = 1024,
Gram route, six gate workers, w_max = 1e-12, eps = 1e-6): one layer on the
GPU; the oracle applies only the central gate, whose four bonds are all at
chi = 1024, and the outputs that depend on that gate alone are compared
(the Schmidt spectra on its two inner bonds and the observables inside its
window).  The oracle runs the dense SVDs of a 5120 x 25600 and a
5120 x 5120 matrix once per module (about a minute of host time); the
FP64, FP32 and split-FP32 theta/gate paths are compared with that one
result, the FP64 path at the FP64 bar and the FP32 paths at 1e-6, with the
per-observable errors printed."""
import numpy as np
import pytest

from gpu_util import note
from oracle import tebd as otebd
from workloads import Model, Trunc, random_mps

pytestmark = pytest.mark.gpu

L, D, CHI, J, TAU = 16, 5, 1024, 6, 0.01
MODEL = Model(L=L, d=D, U=2.0, J=1.0, Jnnn=0.1, K=0.0)


@pytest.fixture(scope="module")
def dense_case():
    B, lam = random_mps(L, D, CHI, seed=0, tau=110.0, bias=150.0)
    assert all(B[i].shape[0] == CHI for i in range(J, J + 4))
    note("full size: oracle gate j=6 (dense SVDs)")
    om = otebd.MPS([b.copy() for b in B], [l.copy() for l in lam])
    otebd.apply_gate(om, J, otebd.GateCache(MODEL)(J, TAU), Trunc(CHI, 1e-12, 1e-6))
    on, oC, oD = otebd.measure(om)
    return B, lam, om, on, oC, oD


def compare(note_tag, n, C, D_, lam_g, om, on, oC, oD):
    win = slice(J, J + 3)
    errs = dict(lam=max(np.abs(lg - om.lam[b]).max() for b, lg in zip((J + 1, J + 2), lam_g)),
                n=float(np.abs(n[win] - on[win]).max()), C=float(np.abs(C[J:J + 2] - oC[J:J + 2]).max()),
                D=float(abs(D_[J] - oD[J])))
    note(f"{note_tag}: errors {errs}, min gap {om.min_gap:.2e}, w {om.w_total:.2e}")
    for b, lg in zip((J + 1, J + 2), lam_g):
        assert len(lg) == len(om.lam[b]), (b, len(lg), len(om.lam[b]))
    return errs


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_bulk_gate_chi1024_sampled(dense_case, prec):
    import paper_2401_05301_amd as pt
    B, lam, om, on, oC, oD = dense_case
    note(f"full size: GPU layer at chi=1024, theta/gate precision {prec}")
    g = pt.MPS.from_tensors(pt.make_model(L, D, MODEL.U, MODEL.J, MODEL.Jnnn, MODEL.K, MODEL.centre()),
                            pt.make_opts(CHI, 1e-12, 1e-6, prec=prec, svd=pt.SVD_GRAM_EIG, workers=6), B, lam)
    g.layer(J % 3, TAU)
    n, C, D_ = g.measure()
    lam_g = [g.lam(J + 1), g.lam(J + 2)]
    g.close()
    errs = compare(f"full size prec={prec}", n, C, D_, lam_g, om, on, oC, oD)
    if prec == 0:
        tol = 1e-10 if om.min_gap >= 1e-8 else max(1e-10, 2 * om.w_total)
    else:
        tol = 1e-6
    assert max(errs.values()) < tol, errs


@pytest.mark.timeout(1200)
def test_bulk_gate_chi1024_sampled_u1():
    """The same check with particle-number sectors (tebd_opts.u1 = 1) on a
    random state of 16 bosons (one per site, so that the central bonds
    reach chi = 1024): the sector SVDs against the oracle's dense
    SVDs of the same gate (spectra compared after sorting, since the
    library groups each bond by particle number)."""
    import paper_2401_05301_amd as pt
    from workloads import random_mps_u1
    B, lam, _ = random_mps_u1(L, D, CHI, L, seed=0, tau=110.0, sigma=2.0, bias=150.0)
    assert all(B[i].shape[0] == CHI for i in range(J, J + 4))
    note(f"full size U(1): bonds {[b.shape[0] for b in B]}")
    g = pt.MPS.from_tensors(pt.make_model(L, D, MODEL.U, MODEL.J, MODEL.Jnnn, MODEL.K, MODEL.centre()),
                            pt.make_opts(CHI, 1e-12, 1e-6, svd=pt.SVD_GRAM_EIG, workers=6, u1=True), B, lam)
    g.layer(J % 3, TAU)
    n, C, D_ = g.measure()
    lam_g = [np.sort(g.lam(J + 1))[::-1], np.sort(g.lam(J + 2))[::-1]]
    g.close()
    note("full size U(1): oracle gate j=6 (dense SVDs)")
    om = otebd.MPS(B, lam)
    otebd.apply_gate(om, J, otebd.GateCache(MODEL)(J, TAU), Trunc(CHI, 1e-12, 1e-6))
    on, oC, oD = otebd.measure(om)
    errs = compare("full size U(1)", n, C, D_, lam_g, om, on, oC, oD)
    tol = 1e-10 if om.min_gap >= 1e-8 else max(1e-10, 2 * om.w_total)
    assert max(errs.values()) < tol, errs
