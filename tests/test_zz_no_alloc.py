"""tebd_diag_svd_noalloc (the truncated SVD with its device buffers in a
file-scope array, for callers that cannot allocate) against tebd_diag_svd
through the C-ABI: two calls in a row, the second on a smaller input (the
array keeps the first call's contents), on both SVD routes."""
import numpy as np
import pytest

from gpu_util import note, rand_c

pytestmark = pytest.mark.gpu


def graded(rng, m, n, decay):
    U, _ = np.linalg.qr(rand_c(rng, m, min(m, n)))
    V, _ = np.linalg.qr(rand_c(rng, n, min(m, n)))
    s = np.exp(-np.arange(min(m, n)) / decay)
    return (U * s) @ V.conj().T


@pytest.mark.parametrize("variant", [0, 1])
def test_noalloc_svd_matches_allocating_entry_point(variant):
    import paper_2401_05301_amd as pt
    rng = np.random.default_rng(17 + variant)
    eps = 1e-12 if variant == 0 else pt.GRAM_EPS_MIN
    for (m, n, chi) in [(200, 320, 64), (48, 30, 12)]:
        A = graded(rng, m, n, decay=max(m, n) / 10.0)
        note(f"noalloc svd variant={variant} m={m} n={n} chi={chi}")
        ref = pt.tebd_diag_svd(A, variant=variant, chi_max=chi, w_max=1e-12, eps=eps)
        got = pt.tebd_diag_svd(A, variant=variant, chi_max=chi, w_max=1e-12, eps=eps, noalloc=True)
        s0, v0, n0, w0, sw0 = ref
        s1, v1, n1, w1, sw1 = got
        assert len(s1) == len(s0) and sw1 == sw0
        assert np.abs(s1 - s0).max() <= 1e-13
        assert abs(n1 - n0) <= 1e-13 * n0 and abs(w1 - w0) <= 1e-15
        # same kernels on the same input: the kept vectors agree to rounding
        assert np.abs(v1 - v0).max() <= 1e-12
        # and they are the singular vectors of A (rows orthonormal, spectrum right)
        sv = np.linalg.svd(A, compute_uv=False)
        assert np.abs(s1 * n1 - sv[:len(s1)]).max() <= 1e-9 * sv[0]


def test_noalloc_svd_rejects_oversize_input():
    import paper_2401_05301_amd as pt
    A = np.zeros((600, 8), dtype=np.complex128)
    with pytest.raises(pt.TebdError) as e:
        pt.tebd_diag_svd(A, variant=0, noalloc=True)
    assert e.value.status == pt.TEBD_EINVAL
    A = np.zeros((300, 300), dtype=np.complex128)
    with pytest.raises(pt.TebdError) as e:
        pt.tebd_diag_svd(A, variant=0, noalloc=True)
    assert e.value.status == pt.TEBD_EINVAL
