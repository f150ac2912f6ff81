"""Full-size check in the configuration bench.py times (d = 5, chi = 1024,
Gram route, four gate workers, w_max = eps = 1e-12): one layer on the GPU;
the oracle applies only the central gate, whose four bonds are all at
chi = 1024, and the outputs that depend on that gate alone are compared
(the Schmidt spectra on its two inner bonds and the observables inside its
window).  The oracle runs the dense SVDs of a 5120 x 25600 and a
5120 x 5120 matrix, so this test takes a few minutes of host time."""
import numpy as np
import pytest

from gpu_util import note
from oracle import tebd as otebd
from workloads import Model, Trunc, random_mps

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(1200)
def test_bulk_gate_chi1024_sampled():
    import paper_2401_05301_amd as pt
    L, d, chi, j, tau = 16, 5, 1024, 6, 0.01
    B, lam = random_mps(L, d, chi, seed=0, tau=110.0, bias=150.0)
    assert all(B[i].shape[0] == chi for i in range(j, j + 4))
    m = Model(L=L, d=d, U=2.0, J=1.0, Jnnn=0.1, K=0.0)
    note("full size: GPU layer at chi=1024")
    g = pt.MPS.from_tensors(pt.make_model(L, d, m.U, m.J, m.Jnnn, m.K, m.centre()),
                            pt.make_opts(chi, 1e-12, 1e-12, svd=pt.SVD_GRAM_EIG, workers=4), B, lam)
    g.layer(j % 3, tau)
    n, C, D = g.measure()
    lam_g = [g.lam(j + 1), g.lam(j + 2)]
    g.close()
    note("full size: oracle gate j=6 (dense SVDs)")
    om = otebd.MPS(B, lam)
    # the Gram route drops singular values below 1e-6 s_0: the oracle applies the same floor
    otebd.apply_gate(om, j, otebd.GateCache(m)(j, tau), Trunc(chi, 1e-12, 1e-6))
    on, oC, oD = otebd.measure(om)
    # Gram route: each Schmidt value to ~1e-8 absolute (SVD #2 inherits the
    # rounding of SVD #1's vectors for small values, ~u s_0^2 / gap); the
    # same bar as for the observables
    for b, lg in zip((j + 1, j + 2), lam_g):
        lo = om.lam[b]
        assert len(lg) == len(lo), (b, len(lg), len(lo))
        assert np.abs(lg - lo).max() < 1e-8, (b, np.abs(lg - lo).max())
    win = slice(j, j + 3)
    assert np.abs(n[win] - on[win]).max() < 1e-8, np.abs(n[win] - on[win]).max()
    assert np.abs(C[j:j + 2] - oC[j:j + 2]).max() < 1e-8
    assert abs(D[j] - oD[j]) < 1e-8


@pytest.mark.timeout(1200)
def test_bulk_gate_chi1024_sampled_u1():
    """The same check with particle-number sectors (tebd_opts.u1 = 1) on a
    random state of 16 bosons (one per site, so that the central bonds
    reach chi = 1024): the sector SVDs against the oracle's dense
    SVDs of the same gate (spectra compared after sorting, since the
    library groups each bond by particle number)."""
    import paper_2401_05301_amd as pt
    from workloads import random_mps_u1
    L, d, chi, j, tau = 16, 5, 1024, 6, 0.01
    B, lam, _ = random_mps_u1(L, d, chi, L, seed=0, tau=110.0, sigma=2.0, bias=150.0)
    assert all(B[i].shape[0] == chi for i in range(j, j + 4))
    m = Model(L=L, d=d, U=2.0, J=1.0, Jnnn=0.1, K=0.0)
    note(f"full size U(1): bonds {[b.shape[0] for b in B]}")
    g = pt.MPS.from_tensors(pt.make_model(L, d, m.U, m.J, m.Jnnn, m.K, m.centre()),
                            pt.make_opts(chi, 1e-12, 1e-12, svd=pt.SVD_GRAM_EIG, workers=4, u1=True), B, lam)
    g.layer(j % 3, tau)
    n, C, D = g.measure()
    lam_g = [np.sort(g.lam(j + 1))[::-1], np.sort(g.lam(j + 2))[::-1]]
    g.close()
    note("full size U(1): oracle gate j=6 (dense SVDs)")
    om = otebd.MPS(B, lam)
    otebd.apply_gate(om, j, otebd.GateCache(m)(j, tau), Trunc(chi, 1e-12, 1e-6))
    on, oC, oD = otebd.measure(om)
    for b, lg in zip((j + 1, j + 2), lam_g):
        lo = om.lam[b]
        assert len(lg) == len(lo), (b, len(lg), len(lo))
        assert np.abs(lg - lo).max() < 1e-8, (b, np.abs(lg - lo).max())
    win = slice(j, j + 3)
    assert np.abs(n[win] - on[win]).max() < 1e-8, np.abs(n[win] - on[win]).max()
    assert np.abs(C[j:j + 2] - oC[j:j + 2]).max() < 1e-8
    assert abs(D[j] - oD[j]) < 1e-8
