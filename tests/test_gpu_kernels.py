"""GPU kernels in isolation, through the diagnostic C-ABI, against NumPy FP64."""
import numpy as np
import pytest

from gpu_util import note, rand_c

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    import paper_2401_05301_amd as pt
    return pt


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (16, 16, 4), (64, 64, 16), (70, 33, 19), (130, 200, 77), (5, 300, 125)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_zgemm_fp64(pt, m, n, k, ta, tb):
    rng = np.random.default_rng(m * 1000 + n * 10 + k + 7 * ta + 3 * tb)
    A = rand_c(rng, *((m, k) if not ta else (k, m)))
    B = rand_c(rng, *((k, n) if not tb else (n, k)))
    note(f"zgemm fp64 m={m} n={n} k={k} ta={ta} tb={tb}")
    C = pt.tebd_diag_zgemm(A, B, ta, tb)
    ref = (A if not ta else A.conj().T) @ (B if not tb else B.conj().T)
    assert np.abs(C - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()) * np.sqrt(k)


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_zgemm_fp64_large_tiles(pt, ta, tb):
    """Shapes large enough for the 128 x 128 tiles, with ragged edges."""
    m, n, k = 2100, 2070, 37
    rng = np.random.default_rng(99 + 2 * ta + tb)
    A = rand_c(rng, *((m, k) if not ta else (k, m)))
    B = rand_c(rng, *((k, n) if not tb else (n, k)))
    ks, rs, cs = rng.random(k), rng.random(m), rng.random(n)
    note(f"zgemm fp64 large m={m} n={n} k={k} ta={ta} tb={tb}")
    C = pt.tebd_diag_zgemm(A, B, ta, tb, k_scale=ks, row_scale=rs, col_scale=cs)
    opA = A if not ta else A.conj().T
    opB = B if not tb else B.conj().T
    ref = rs[:, None] * ((opA * ks[None, :]) @ opB) * cs[None, :]
    assert np.abs(C - ref).max() <= 1e-13 * np.abs(ref).max() * np.sqrt(k)


@pytest.mark.parametrize("m,k,ta", [(70, 19, 0), (130, 40, 1), (2100, 33, 0), (2100, 33, 1)])
def test_zgemm_hermitian_output(pt, m, k, ta):
    """Gram products computed on the lower tiles and mirrored."""
    rng = np.random.default_rng(m + k + ta)
    X = rand_c(rng, *((m, k) if not ta else (k, m)))
    rs = rng.random(m) + 0.5
    note(f"zgemm herm m={m} k={k} ta={ta}")
    # op(A) = X (or X^+ when stored transposed), op(B) = op(A)^+
    C = pt.tebd_diag_zgemm(X, X, ta, 1 - ta, row_scale=rs, col_scale=rs, herm=True)
    opA = X if not ta else X.conj().T
    ref = rs[:, None] * (opA @ opA.conj().T) * rs[None, :]
    assert np.abs(C - ref).max() <= 1e-13 * np.abs(ref).max() * np.sqrt(k)
    assert np.abs(C - C.conj().T).max() <= 1e-13 * np.abs(ref).max()


def test_zgemm_scalings(pt):
    rng = np.random.default_rng(3)
    m, n, k = 45, 67, 29
    A, B = rand_c(rng, m, k), rand_c(rng, k, n)
    ks, rs, cs = rng.random(k), rng.random(m), rng.random(n)
    note("zgemm scalings")
    C = pt.tebd_diag_zgemm(A, B, k_scale=ks, row_scale=rs, col_scale=cs)
    ref = rs[:, None] * (A @ np.diag(ks) @ B) * cs[None, :]
    assert np.abs(C - ref).max() < 1e-12


@pytest.mark.parametrize("prec,tol", [(1, 3e-5), (2, 3e-6)])
def test_zgemm_reduced_precision(pt, prec, tol):
    rng = np.random.default_rng(11)
    A, B = rand_c(rng, 96, 125), rand_c(rng, 125, 80)
    note(f"zgemm prec={prec}")
    C = pt.tebd_diag_zgemm(A, B, prec=prec)
    ref = A @ B
    rel = np.abs(C - ref).max() / np.abs(ref).max()
    assert rel < tol, rel
    if prec == 2:
        C1 = pt.tebd_diag_zgemm(A, B, prec=1)
        assert rel < np.abs(C1 - ref).max() / np.abs(ref).max()


def graded_matrix(rng, m, n, decay):
    r = min(m, n)
    U, _ = np.linalg.qr(rand_c(rng, m, r))
    V, _ = np.linalg.qr(rand_c(rng, n, r))
    s = np.exp(-np.arange(r) / decay)
    return (U * s) @ V.conj().T, s


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("m,n", [(3, 9), (12, 7), (40, 100), (100, 40), (257, 130)])
def test_svd_spectrum_and_subspace(pt, variant, m, n):
    rng = np.random.default_rng(m + 7 * n + variant)
    A, s_true = graded_matrix(rng, m, n, decay=max(m, n) / 12.0)
    note(f"svd variant={variant} m={m} n={n}")
    eps = 1e-12 if variant == 0 else 1e-6   # the Gram route takes eps >= 1e-6
    s, vh, nrm, w, sweeps = pt.tebd_diag_svd(A, variant=variant, w_max=1e-10, eps=eps)
    _, s_ref, vh_ref = np.linalg.svd(A, full_matrices=False)
    k = len(s)
    assert sweeps >= 1
    # truncation decision identical to the rule applied to the exact spectrum
    tot = np.sum(s_ref ** 2)
    tails = np.cumsum((s_ref ** 2)[::-1])[::-1]
    kw = next(kk for kk in range(len(s_ref) + 1) if (tails[kk] if kk < len(s_ref) else 0.0) <= 1e-10 * tot)
    ke = int(np.sum(s_ref > eps * s_ref[0]))
    assert k == max(1, min(kw, ke))
    tol = 1e-12 if variant == 0 else 1e-9
    assert np.abs(s * nrm - s_ref[:k]).max() < tol * s_ref[0]
    # kept right singular vectors span the same subspace (rows orthonormal)
    assert np.abs(vh @ vh.conj().T - np.eye(k)).max() < (1e-12 if variant == 0 else 1e-6)
    P = vh.conj().T @ vh
    Pr = vh_ref[:k].conj().T @ vh_ref[:k]
    assert np.abs(P - Pr).max() < (1e-10 if variant == 0 else 1e-5)


def test_svd_rank_deficient_and_chi_cap(pt):
    rng = np.random.default_rng(5)
    A = rand_c(rng, 60, 4) @ rand_c(rng, 4, 90)   # rank 4
    note("svd rank deficient")
    s, vh, nrm, w, _ = pt.tebd_diag_svd(A, variant=0, w_max=0.0, eps=1e-12)
    assert len(s) == 4
    assert abs(np.sum(s ** 2) - 1) < 1e-14
    s2, vh2, _, w2, _ = pt.tebd_diag_svd(A, variant=0, chi_max=2)
    sr = np.linalg.svd(A, compute_uv=False)
    assert len(s2) == 2
    assert abs(w2 - np.sum(sr[2:] ** 2) / np.sum(sr ** 2)) < 1e-13


@pytest.mark.parametrize("m,n,chi", [(1100, 1800, 64), (1800, 1100, 48), (1280, 3000, 128), (400, 900, 64)])
def test_gram_subspace_topk(pt, m, n, chi):
    """Gram route with subspace iteration (chi_max well below min(m, n),
    at least 1024 rows), and the direct solve below that size."""
    rng = np.random.default_rng(m + n + chi)
    A, s_true = graded_matrix(rng, m, n, decay=chi / 4.0)
    note(f"gram subspace m={m} n={n} chi={chi}")
    s, vh, nrm, w, sweeps = pt.tebd_diag_svd(A, variant=1, chi_max=chi, w_max=1e-14, eps=1e-6)
    _, s_ref, vh_ref = np.linalg.svd(A, full_matrices=False)
    k = len(s)
    assert k == chi
    assert np.abs(s * nrm - s_ref[:k]).max() < 1e-9 * s_ref[0]
    tot = np.sum(s_ref ** 2)
    assert abs(w - np.sum(s_ref[k:] ** 2) / tot) < 1e-12
    P = vh.conj().T @ vh
    Pr = vh_ref[:k].conj().T @ vh_ref[:k]
    assert np.abs(P - Pr).max() < 1e-6


@pytest.mark.parametrize("m,n,rank,chi", [(1100, 1300, 150, 128), (1300, 1100, 1, 64), (1100, 2600, 300, 256)])
def test_gram_subspace_rank_deficient(pt, m, n, rank, chi):
    """Subspace route on a Gram matrix whose rank lies below the subspace
    width (as for an identity gate on a state of exact bond dimension), with
    a steep spectrum inside the rank."""
    rng = np.random.default_rng(m + n + rank)
    U, _ = np.linalg.qr(rand_c(rng, m, rank))
    V, _ = np.linalg.qr(rand_c(rng, n, rank))
    s_true = np.exp(-np.arange(rank) / (rank / 12.0))
    A = (U * s_true) @ V.conj().T
    note(f"gram subspace rank-deficient m={m} n={n} rank={rank} chi={chi}")
    s, vh, nrm, w, sweeps = pt.tebd_diag_svd(A, variant=1, chi_max=chi, w_max=1e-14, eps=1e-6)
    k = len(s)
    sv = np.sort(s_true)[::-1]
    assert k == min(chi, rank) or (k < min(chi, rank) and sv[k] <= 1e-6 * sv[0])
    assert np.abs(s * nrm - sv[:k]).max() < 1e-9 * sv[0]
    # the Gram route resolves a singular vector to ~u / (relative gap * s_i^2):
    # near-orthonormal rows, exact to rounding once weighted by the values
    E = vh @ vh.conj().T - np.eye(k)
    assert np.abs(E).max() < 1e-4
    sk = sv[:k]
    assert np.abs(sk[:, None] * E * sk[None, :]).max() < 1e-12
    # the kept rows lie in the row space of A
    assert np.linalg.norm(vh - (vh @ V) @ V.conj().T) < 1e-6 * np.sqrt(k)
