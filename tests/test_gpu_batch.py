"""Batched evaluation: a workspace of several instances (the same model at
several thetas, or models of different sizes) must give, instance by
instance, exactly the results of single-instance workspaces (same kernels,
same reduction orders), and those match the CPU oracle.  Also: Q_p assembled
just in time gives the same log-determinant as Q_p stored in full, and a
replayed HIP graph gives the eager results on every replay."""
import numpy as np
import pytest

import workloads as W
from oracle import fobj as OF

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_06938_amd import dalia
    dalia.lib()
    return dalia


def _single(D, wl, theta, selinv=False):
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=selinv)
    f, parts, info = ws.fobj(theta)
    out = [f.cpu().numpy(), parts.cpu().numpy(), info.cpu().numpy()]
    if selinv:
        out.append(ws.selinv().cpu().numpy())
    torch.cuda.synchronize()
    return out


def test_fd_batch_equals_single_calls(D):
    """2*dim+1 central-difference points of the tiny univariate workload in
    one batch (Eq. 10 stencil), bitwise equal to one-by-one evaluation."""
    wl = W.config0()
    h = 1e-3
    pts = [wl.theta]
    for i in range(wl.dim_theta):
        e = np.zeros(wl.dim_theta)
        e[i] = h
        pts += [wl.theta + e, wl.theta - e]
    pts = np.stack(pts)
    model = D.Model.from_workload(wl)
    ws = D.Workspace([model] * len(pts), selinv=True)
    f, parts, info = ws.fobj(pts)
    var = ws.selinv().cpu().numpy()
    torch.cuda.synchronize()
    f = f.cpu().numpy()
    for k, th in enumerate(pts):
        fs, ps, _, vs = _single(D, wl, th, selinv=True)
        assert f[k] == fs[0], k
        assert np.array_equal(var[k * wl.N:(k + 1) * wl.N], vs)
    ref = OF.fobj(wl, pts[3])
    p = parts.cpu().numpy()[3]
    assert abs(f[3] - ref) <= 1e-10 * (abs(p[1]) + abs(p[2]))


def test_more_thetas_than_instances(D):
    wl = W.config0()
    model = D.Model.from_workload(wl)
    ws = D.Workspace([model] * 3)
    rng = np.random.default_rng(5)
    th = wl.theta[None] + 0.05 * rng.standard_normal((7, wl.dim_theta))
    f, _, _ = ws.fobj(th)
    f = f.cpu().numpy()
    for k in range(7):
        assert f[k] == _single(D, wl, th[k])[0][0]


def test_uneven_batch(D):
    wls = [W.scaled("u0", 6, 5, 1, 2, 60, seed=1), W.scaled("u1", 5, 3, 3, 1, 40, seed=2),
           W.scaled("u2", 9, 4, 1, 3, 90, seed=3), W.scaled("u3", 4, 7, 2, 2, 30, seed=4)]
    models = [D.Model.from_workload(w) for w in wls]
    ws = D.Workspace(models, selinv=True)
    thetas = np.concatenate([w.theta + 0.02 for w in wls])
    f, parts, info = ws.fobj(thetas)
    var = ws.selinv().cpu().numpy()
    torch.cuda.synchronize()
    f = f.cpu().numpy()
    off = 0
    for k, w in enumerate(wls):
        fs, ps, _, vs = _single(D, w, w.theta + 0.02, selinv=True)
        assert f[k] == fs[0], k
        assert np.array_equal(var[off:off + w.N], vs)
        off += w.N
        ref = OF.fobj_parts(w, w.theta + 0.02)
        scale = abs(ref["logdet_p"]) + abs(ref["logdet_c"])
        assert abs(f[k] - ref["f"]) <= 1e-10 * scale


def test_qp_ring_equals_full_storage(D):
    wl = W.scaled("ring", 8, 6, 1, 2, 80, seed=6)
    model = D.Model.from_workload(wl)
    a = D.Workspace(model)
    b = D.Workspace(model, keep_qp=True)
    fa, pa, _ = a.fobj(wl.theta)
    fb, pb, _ = b.fobj(wl.theta)
    torch.cuda.synchronize()
    assert pa.cpu().numpy()[0, 1] == pb.cpu().numpy()[0, 1]
    assert fa.item() == fb.item()


def test_graph_replays_match_eager(D):
    wl = W.scaled("graph", 7, 5, 1, 2, 70, seed=7)
    model = D.Model.from_workload(wl)
    eager = D.Workspace([model] * 2)
    graph = D.Workspace([model] * 2, graph=True)
    rng = np.random.default_rng(8)
    for rep in range(4):
        th = wl.theta[None] + 0.05 * rng.standard_normal((2, wl.dim_theta))
        fg, pg, _ = graph.fobj(th)
        x = torch.randn(1000, device="cuda").sum()   # eager work in between
        torch.cuda.synchronize()
        fe, pe, _ = eager.fobj(th)
        torch.cuda.synchronize()
        assert np.array_equal(fg.cpu().numpy(), fe.cpu().numpy()), rep
        assert np.array_equal(pg.cpu().numpy(), pe.cpu().numpy()), rep
        del x


def test_autotuned_tiles_give_identical_results(D, tmp_path):
    """Both GEMM tile sizes sum each output over the same k sequence (extra
    terms are exact zeros), so a tuned workspace whose products are too short
    to split (k <= 512) reproduces the default one bit for bit; the cache
    file is written and reused."""
    wl = W.scaled("tune", 12, 4, 1, 2, 200, seed=9)
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True)
    f0, p0, _ = ws.fobj(wl.theta)
    v0 = ws.selinv().cpu().numpy()
    cache = str(tmp_path / "tiles.txt")
    counts = ws.autotune(cache)
    assert counts["tile64"] + counts["tile128"] > 0
    f1, p1, _ = ws.fobj(wl.theta)
    v1 = ws.selinv().cpu().numpy()
    torch.cuda.synchronize()
    assert f0.item() == f1.item()
    assert np.array_equal(v0, v1)
    lines = open(cache).read().splitlines()
    assert lines and all(l.rsplit(" ", 1)[1] in ("64", "128") for l in lines)
    ws2 = D.Workspace(model, selinv=True)
    assert ws2.autotune(cache) == counts   # read back from the cache


def test_autotune_with_split_candidates(D, tmp_path):
    """Blocks of 576 (k > 512): the tuner may also choose split k (pieces of
    512 or 256), which sums the k pieces separately, so results agree with
    the default workspace to rounding; a second workspace reads every choice
    back from the cache."""
    wl = W.scaled("tune_split", 24, 3, 1, 2, 400, seed=4)
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True)
    f0, p0, _ = ws.fobj(wl.theta)
    v0 = ws.selinv().cpu().numpy()
    cache = str(tmp_path / "tiles.txt")
    counts = ws.autotune(cache)
    f1, p1, _ = ws.fobj(wl.theta)
    v1 = ws.selinv().cpu().numpy()
    torch.cuda.synchronize()
    assert abs(f1.item() - f0.item()) <= 1e-12 * abs(f0.item())
    np.testing.assert_allclose(p1.cpu().numpy(), p0.cpu().numpy(), rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(v1, v0, rtol=1e-10)
    lines = open(cache).read().splitlines()
    assert lines and all(l.rsplit(" ", 1)[1] in ("64", "128", "64s", "128s", "64s256", "128s256")
                         for l in lines)
    ws2 = D.Workspace(model, selinv=True)
    assert ws2.autotune(cache) == counts
    f2, _, _ = ws2.fobj(wl.theta)
    torch.cuda.synchronize()
    assert f2.item() == f1.item()
