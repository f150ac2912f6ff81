"""Error contract of the C-ABI on the GPU: an SVD that does not converge
within max_sweeps returns ENOCONV and leaves the handle refusing further
evolution, measurement and checkpoints (ESTATE), on every SVD route, with one gate worker
and with several, and with fused layers.  The sweep limit is set from the host, so every kernel
still runs its normal, bounded course."""
import pytest

from gpu_util import note
from workloads import Model, random_mps, random_mps_u1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    import paper_2401_05301_amd as pt
    return pt


CASES = [
    # (svd route, U(1) sectors, gate workers, fused layers)
    (0, False, 1, False), (0, False, 3, False), (1, False, 1, False), (1, False, 3, False), (0, True, 1, False),
    (1, True, 3, False), (0, False, 0, True),
]


@pytest.mark.parametrize("svd,u1,workers,fuse", CASES)
def test_unconverged_svd_marks_handle(pt, svd, u1, workers, fuse):
    note(f"ENOCONV svd={svd} u1={u1} workers={workers} fuse={fuse}")
    L, d, chi = 12, 3, 24
    if u1:
        B, lam, _ = random_mps_u1(L, d, chi, L // 2, seed=4, tau=8.0)
    else:
        B, lam = random_mps(L, d, chi, seed=4)
    m = Model(L=L, d=d, U=2.0, J=1.0, Jnnn=0.1, K=0.01)
    opts = pt.make_opts(chi, 1e-12, 1e-12 if svd == 0 else 1e-6, svd=svd, max_sweeps=1, workers=workers, u1=u1,
                        fuse=fuse)
    g = pt.MPS.from_tensors(pt.make_model(m.L, m.d, m.U, m.J, m.Jnnn, m.K, m.centre()), opts, B, lam)
    with pytest.raises(pt.TebdError) as e:
        g.layer(0, 0.05)
    assert e.value.status == pt.TEBD_ENOCONV
    for call in (lambda: g.layer(1, 0.05), g.measure, lambda: g.step(0.05), g.checkpoint):
        with pytest.raises(pt.TebdError) as e:
            call()
        assert e.value.status == pt.TEBD_ESTATE
    g.close()


def test_converged_handle_still_usable(pt):
    """The same state with the default sweep limit evolves and measures."""
    note("default max_sweeps evolves")
    L, d, chi = 12, 3, 24
    B, lam = random_mps(L, d, chi, seed=4)
    m = Model(L=L, d=d, U=2.0, J=1.0, Jnnn=0.1, K=0.01)
    g = pt.MPS.from_tensors(pt.make_model(m.L, m.d, m.U, m.J, m.Jnnn, m.K, m.centre()),
                            pt.make_opts(chi, 1e-12, 1e-12, workers=3), B, lam)
    g.layer(0, 0.05)
    n, C, D = g.measure()
    assert len(n) == L
    g.close()
