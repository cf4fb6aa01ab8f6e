"""GPU unit tests of the dense FP64 building blocks against numpy/LAPACK on
the host (random inputs; sizes span several 64x64 tiles and ragged edges)."""
import numpy as np
import pytest
import scipy.linalg as sla

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_06938_amd import dalia
    dalia.lib()
    return dalia


def _dev(x):
    return torch.from_numpy(np.asfortranarray(x)).cuda()


def _colmajor(x):
    t = torch.from_numpy(np.ascontiguousarray(x.T)).cuda()
    return t.T


@pytest.mark.parametrize("M,N,K,ta,tb", [
    (64, 64, 64, 0, 1), (130, 70, 33, 0, 0), (128, 192, 100, 1, 0),
    (65, 200, 17, 1, 1), (256, 256, 256, 0, 1), (1, 1, 1, 0, 0),
    # vector-staged operands: even extents, 16-byte aligned columns; odd and
    # even chunk counts, partial edge tiles inside the vector path
    (384, 320, 272, 0, 1), (320, 384, 208, 1, 0), (130, 66, 48, 1, 1),
    (66, 130, 32, 0, 0), (192, 64, 16, 1, 1),
])
def test_dgemm_matches_numpy(D, M, N, K, ta, tb):
    rng = np.random.default_rng(M * 7 + N)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    want = 0.7 * ((A.T if ta else A) @ (B.T if tb else B)) - 1.3 * C0
    Ad, Bd, Cd = _colmajor(A), _colmajor(B), _colmajor(C0)
    D.dgemm(Ad, Bd, Cd, transa=bool(ta), transb=bool(tb), alpha=0.7, beta=-1.3)
    got = Cd.cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_dgemm_lower_touches_only_lower(D):
    rng = np.random.default_rng(3)
    n, k = 150, 40
    A = rng.standard_normal((n, k))
    C0 = rng.standard_normal((n, n))
    Cd = _colmajor(C0)
    Ad = _colmajor(A)
    D.dgemm(Ad, Ad, Cd, transb=True, lower=True, alpha=-1.0, beta=1.0)
    got = Cd.cpu().numpy()
    want = C0 - A @ A.T
    il = np.tril_indices(n)
    iu = np.triu_indices(n, 1)
    np.testing.assert_allclose(got[il], want[il], rtol=1e-12, atol=1e-11)
    assert np.array_equal(got[iu], C0[iu])


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n))
    return B @ B.T / n + np.eye(n)


@pytest.mark.parametrize("n", [64, 128, 320, 1024])
def test_dpotrf_matches_lapack(D, n):
    A = _spd(n, n)
    Ad = _colmajor(A)
    ld, info = D.dpotrf(Ad)
    L = sla.cholesky(A, lower=True)
    assert int(info.item()) == 0
    assert abs(ld.item() - 2 * np.sum(np.log(np.diag(L)))) < 1e-11 * n
    got = np.tril(Ad.cpu().numpy())
    np.testing.assert_allclose(got, L, rtol=1e-10, atol=1e-12)
    assert np.all(np.triu(Ad.cpu().numpy(), 1) == 0)


@pytest.mark.parametrize("n", [64, 192, 640])
def test_dpotrf_inverse(D, n):
    A = _spd(n, 11 + n)
    Ad = _colmajor(A)
    ld, info = D.dpotrf(Ad, inverse=True)
    L = sla.cholesky(A, lower=True)
    G = sla.solve_triangular(L, np.eye(n), lower=True)
    got = Ad.cpu().numpy()
    np.testing.assert_allclose(got, G, rtol=1e-9, atol=1e-11)


def test_dpotrf_reports_first_bad_pivot(D):
    n = 192
    A = _spd(n, 5)
    A[130, 130] = -5.0   # not SPD; LAPACK reports the first failing column
    Ad = _colmajor(A)
    _, info = D.dpotrf(Ad)
    try:
        sla.cholesky(A, lower=True)
        pytest.fail("LAPACK accepted a non-SPD matrix")
    except np.linalg.LinAlgError:
        pass
    # lapack's dpotrf info (1-based) for the same matrix
    _, linfo = sla.lapack.dpotrf(A, lower=1)
    assert int(info.item()) == linfo
