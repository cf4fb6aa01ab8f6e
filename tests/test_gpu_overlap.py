"""fobj_selinv_eval: f_obj and the marginal variances in one call, the solve
running on a second stream while the selected inversion runs on the caller's
stream.  The launches and their inputs are those of fobj_eval followed by
bta_selinv, so the results must agree bit for bit; checked for a single
model, a batch of two thetas and a mixed-precision workspace, and on two
calls in a row (the second with other thetas)."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_06938_amd import dalia
    dalia.lib()
    return dalia


@pytest.mark.parametrize("batch,mixed", [(1, False), (2, False), (1, True)])
def test_overlapped_matches_sequential(D, batch, mixed):
    wl = W.scaled("overlap", 14, 5, 3, 2, 300, seed=8)
    print(f"batch {batch} mixed {mixed} N={wl.N}", flush=True)
    model = D.Model.from_workload(wl)
    ws = D.Workspace([model] * batch, selinv=True, mixed=mixed)
    rng = np.random.default_rng(3)
    for call in range(2):
        th = wl.theta[None] + 0.05 * rng.standard_normal((batch, wl.dim_theta))
        f1, p1, i1, v1 = ws.fobj_selinv(th)
        torch.cuda.synchronize()
        r1 = (f1.cpu().numpy().copy(), p1.cpu().numpy().copy(), i1.cpu().numpy().copy(),
              v1.cpu().numpy().copy())
        f0, p0, i0 = ws.fobj(th)
        v0 = ws.selinv()
        torch.cuda.synchronize()
        assert (i0.cpu().numpy() == 0).all()
        assert np.array_equal(r1[0], f0.cpu().numpy()), call
        assert np.array_equal(r1[1], p0.cpu().numpy()), call
        assert np.array_equal(r1[2], i0.cpu().numpy()), call
        assert np.array_equal(r1[3], v0.cpu().numpy()), call


def test_overlapped_requires_selinv_workspace(D):
    wl = W.scaled("overlap_nosel", 10, 3, 1, 2, 100, seed=2)
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model)
    with pytest.raises(D.DaliaError):
        ws.fobj_selinv(wl.theta)
