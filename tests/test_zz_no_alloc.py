"""dl_dpotrf_noalloc (the dense Cholesky for callers that cannot allocate)
against dl_dpotrf: the same kernels on the same descriptors, so L (or L^-1),
log|A| and info agree bit for bit.  Two calls in a row, the second with a
smaller matrix, so that the shared scratch array's leftovers from the first
call must not leak into the second; plus a matrix with a bad pivot."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_06938_amd import dalia
    dalia.lib()
    return dalia


def spd(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n + 8))
    return X @ X.T / n + 0.5 * np.eye(n)


def both(D, A, inverse):
    dev = torch.device("cuda")
    A0 = D.fortran(torch.tensor(A, dtype=torch.float64, device=dev))
    A1 = A0.clone()
    ld0, info0 = D.dpotrf(A0, inverse=inverse)
    ld1 = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
    info1 = torch.full((1,), -7, dtype=torch.int64, device=dev)
    D.dpotrf_noalloc(A1, ld1, info1, inverse=inverse)
    torch.cuda.synchronize()
    return (A0.cpu().numpy(), ld0.item(), info0.item()), (A1.cpu().numpy(), ld1.item(),
                                                          info1.item())


@pytest.mark.parametrize("inverse", [False, True])
def test_noalloc_matches_allocating_entry_point(D, inverse):
    for call, n in enumerate((2048, 320)):  # second call smaller
        print(f"call {call} n={n} inverse={inverse}", flush=True)
        A = spd(n, 10 + call)
        (L0, ld0, i0), (L1, ld1, i1) = both(D, A, inverse)
        assert i0 == 0 and i1 == 0
        assert np.array_equal(np.tril(L0), np.tril(L1)), (call, n)
        assert ld0 == ld1, (call, ld0, ld1)
        # and both are the Cholesky factor (or its inverse) of A
        want = np.linalg.slogdet(A)[1]
        assert abs(ld1 - want) <= 1e-10 * abs(want)
        Lref = np.linalg.cholesky(A)
        got = np.linalg.inv(np.tril(L1)) if inverse else np.tril(L1)
        np.testing.assert_allclose(got, Lref, rtol=0, atol=1e-9 * np.abs(Lref).max())


def test_noalloc_reports_the_first_bad_pivot(D):
    n = 384
    A = spd(n, 3)
    A[200, 200] = -1.0  # the leading 200 x 200 block stays SPD
    (_, _, i0), (_, _, i1) = both(D, A, False)
    assert i0 == 201 and i1 == 201


def test_noalloc_rejects_sizes_beyond_its_scratch(D):
    dev = torch.device("cuda")
    ld = torch.empty(1, dtype=torch.float64, device=dev)
    info = torch.empty(1, dtype=torch.int64, device=dev)
    for n in (D.DPOTRF_NOALLOC_MAX_N + 64, 40):  # too large; not a multiple of 64
        A = D.fortran(torch.zeros((n, n), dtype=torch.float64, device=dev))
        with pytest.raises(D.DaliaError):
            D.dpotrf_noalloc(A, ld, info)
