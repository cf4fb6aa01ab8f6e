"""The C-ABI boundary beyond fobj_eval, through the ctypes binding:

  * bta_solve with caller right-hand sides (several at once), FP64
    refinement to a tolerance and the DL_ENOTCONV report when a refinement
    cannot reach it, against the oracle's dense Q_c;
  * dl_permute / dl_unpermute against the oracle's permutation;
  * dl_ws_set_block: a caller-modified BTA matrix factored, solved and
    inverted against the oracle's dense routines, and planted non-positive
    pivots in a diagonal block (first, chain A, chain B, middle block, last)
    and in the tip, reported by bta_factor as 1 + their BTA row, in both
    elimination orders;
  * dl_ws_estimate_bytes / dl_ws_create_budget / dl_plan_waves against the
    bytes a created workspace reports;
  * mixed-precision refinement: batch, single and graph-replayed
    evaluations agree bit for bit and the refined mean meets 1e-12.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fobj as OF
from oracle import model as OM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_06938_amd import dalia
    dalia.lib()
    return dalia


def dense_qc_bta(wl, theta):
    """The oracle's Q_c as a dense matrix in BTA order."""
    ref = OF.fobj_parts(wl, theta, return_factors=True)
    perm = OM.bta_permutation(wl.nv, wl.ns, wl.nt, wl.nr)
    Q = ref["Qc"].toarray()[np.ix_(perm, perm)]
    return Q, ref, perm


def cuda(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("mixed", [False, True])
def test_solve_caller_rhs_with_refinement(D, mixed):
    wl = W.scaled("solve", 8, 6, 3, 2, 60, seed=31)
    Q, ref, perm = dense_qc_bta(wl, wl.theta)
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, mixed=mixed, two_sided=True)
    ws.assemble(wl.theta)
    ld, info = ws.factor()
    rng = np.random.default_rng(2)
    R = rng.standard_normal((3, wl.N))
    want = np.linalg.solve(Q, R.T).T
    for refine_max in (0, 6):
        x = cuda(R)
        x, conv = ws.solve(x, refine_max=refine_max, return_converged=True)
        torch.cuda.synchronize()
        got = x.cpu().numpy()
        res = np.linalg.norm(R - got @ Q.T, axis=1) / np.linalg.norm(R, axis=1)
        if refine_max > 0 or not mixed:
            assert conv
            assert np.all(res <= 1e-12), (refine_max, res)
            np.testing.assert_allclose(got, want, rtol=0,
                                       atol=1e-9 * np.abs(want).max())
        else:
            assert np.all(res <= 1e-3), res  # one FP32-factor solve, unrefined
    # a tolerance no refinement reaches: DL_ENOTCONV, x still written
    x = cuda(R[0])
    x, conv = ws.solve(x, refine_max=2, refine_tol=1e-300, return_converged=True)
    torch.cuda.synchronize()
    assert not conv
    np.testing.assert_allclose(x.cpu().numpy(), want[0], rtol=0,
                               atol=1e-6 * np.abs(want).max())
    # the default solve of the assembled right-hand side gives the mean
    ws.assemble(wl.theta)
    ws.factor()
    mu = ws.solve()
    torch.cuda.synchronize()
    np.testing.assert_allclose(mu.cpu().numpy(), ref["mu"][perm], rtol=0,
                               atol=1e-9 * np.abs(ref["mu"]).max())


def test_solve_rejects_bad_arguments(D):
    wl = W.scaled("solve_bad", 6, 3, 1, 1, 40, seed=3)
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model)
    x = torch.zeros(wl.N, dtype=torch.float64, device="cuda")
    with pytest.raises(D.DaliaError):  # before any factorisation
        ws.solve(x)
    ws.assemble(wl.theta)
    ws.factor()
    L = D.lib()
    for nrhs, rmax, tol in ((0, 0, 0.0), (1, 101, 1e-12), (1, 2, -1.0), (1, 2, float("nan"))):
        assert L.bta_solve(ws.h, D._ptr(x), nrhs, rmax, tol, D._stream()) == 1


@pytest.mark.parametrize("nv", [1, 3])
def test_permute_matches_oracle(D, nv):
    wl = W.scaled("perm", 5, 4, nv, 2, 30, seed=4)
    model = D.Model.from_workload(wl)
    perm = OM.bta_permutation(wl.nv, wl.ns, wl.nt, wl.nr)
    X = np.random.default_rng(1).standard_normal((2, wl.N))
    xb = model.permute(cuda(X))
    torch.cuda.synchronize()
    assert np.array_equal(xb.cpu().numpy(), X[:, perm])
    back = model.unpermute(xb)
    torch.cuda.synchronize()
    assert np.array_equal(back.cpu().numpy(), X)
    one = model.permute(cuda(X[0]))
    torch.cuda.synchronize()
    assert np.array_equal(one.cpu().numpy(), X[0, perm])


def test_set_block_modified_matrix_against_dense(D):
    """A caller-modified BTA matrix: D_2 gets +1 on its diagonal and the
    tip +0.5; log|Q|, the solve and diag(Q^-1) against dense numpy."""
    wl = W.scaled("setb", 7, 5, 1, 2, 80, seed=5)
    Q, ref, perm = dense_qc_bta(wl, wl.theta)
    model = D.Model.from_workload(wl)
    b, a = wl.b, wl.a
    for two in (False, True):
        ws = D.Workspace(model, selinv=True, two_sided=two)
        ws.assemble(wl.theta, D.DL_QC)
        Dt = ws.get_block(D.DL_QC, 0, 2).cpu().numpy()
        np.testing.assert_allclose(np.tril(Dt), np.tril(Q[2 * b:3 * b, 2 * b:3 * b]),
                                   rtol=0, atol=1e-12 * np.abs(Q).max())
        ws.set_block(D.DL_QC, 0, 2, cuda(Dt + np.eye(b)))
        tip = ws.get_block(D.DL_QC, 3, 0).cpu().numpy()
        ws.set_block(D.DL_QC, 3, 0, cuda(tip + 0.5 * np.eye(a)))
        Q2 = Q.copy()
        Q2[2 * b:3 * b, 2 * b:3 * b] += np.eye(b)
        Q2[-a:, -a:] += 0.5 * np.eye(a)
        ld, info = ws.factor(D.DL_QC)
        torch.cuda.synchronize()
        assert info.cpu().tolist() == [0]
        want = np.linalg.slogdet(Q2)[1]
        assert abs(ld.item() - want) <= 1e-10 * abs(want)
        r = np.random.default_rng(6).standard_normal(wl.N)
        x = ws.solve(cuda(r), refine_max=0)
        var = ws.selinv()
        torch.cuda.synchronize()
        xs = np.linalg.solve(Q2, r)
        np.testing.assert_allclose(x.cpu().numpy(), xs, rtol=0, atol=1e-9 * np.abs(xs).max())
        np.testing.assert_allclose(var.cpu().numpy(), np.diag(np.linalg.inv(Q2)), rtol=1e-9)


@pytest.mark.parametrize("two_sided", [False, True])
def test_planted_bad_pivot_reports_bta_row(D, two_sided):
    wl = W.scaled("pivot", 9, 7, 1, 3, 140, seed=17)  # b = 81 (ragged), nt = 7
    model = D.Model.from_workload(wl)
    b = wl.b
    ws = D.Workspace(model, two_sided=two_sided)
    mid = (wl.nt + 1) // 2
    cases = [(0, 0), (1, 37), (mid, 64), (wl.nt - 2, 80), (wl.nt - 1, 5)]
    for t, r in cases:
        ws.assemble(wl.theta, D.DL_QC)
        Dt = ws.get_block(D.DL_QC, 0, t).cpu().numpy().copy()
        Dt[r, r] = -1.0  # the leading r x r part stays positive definite
        ws.set_block(D.DL_QC, 0, t, cuda(Dt))
        ld, info = ws.factor(D.DL_QC)
        torch.cuda.synchronize()
        print(f"two_sided={two_sided} t={t} r={r} info={info.item()}", flush=True)
        assert info.item() == t * b + r + 1, (t, r, info.item())
    # the tip: row nt*b + r
    ws.assemble(wl.theta, D.DL_QC)
    tip = ws.get_block(D.DL_QC, 3, 0).cpu().numpy().copy()
    tip[1, 1] = -2.0
    ws.set_block(D.DL_QC, 3, 0, cuda(tip))
    ld, info = ws.factor(D.DL_QC)
    torch.cuda.synchronize()
    assert info.item() == wl.nt * b + 1 + 1
    # set_block needs an assembled, unfactored matrix
    with pytest.raises(D.DaliaError):
        ws.set_block(D.DL_QC, 3, 0, cuda(tip))


def test_memory_estimate_budget_and_waves(D):
    wls = [W.scaled("m1", 10, 6, 1, 2, 80, seed=1), W.scaled("m3", 8, 5, 3, 2, 40, seed=2),
           W.scaled("m1b", 14, 9, 1, 2, 100, seed=3)]
    models = [D.Model.from_workload(w) for w in wls]
    for kw in ({}, {"selinv": True, "two_sided": True}, {"mixed": True, "fold_inverse": True}):
        est = D.estimate_bytes(models, **kw)
        ws = D.Workspace(models, **kw)
        got = ws.nbytes
        del ws
        print(kw, est, got, flush=True)
        assert est <= got <= est + D.DL_WAVE_RESERVE, (kw, est, got)
    est = D.estimate_bytes(models)
    with pytest.raises(D.DaliaError) as e:
        D.Workspace(models, hbm_budget=est - 1)
    assert e.value.code == 2
    ws = D.Workspace(models, hbm_budget=est)
    del ws
    per = [D.estimate_bytes([m]) for m in models]
    budget = max(per) + D.DL_WAVE_RESERVE + 1024
    waves = D.plan_waves(models, budget)
    assert sorted(k for w in waves for k in w) == [0, 1, 2]
    for w in waves:
        assert D.estimate_bytes([models[k] for k in w]) + D.DL_WAVE_RESERVE <= budget + 1024 * len(w)
    assert len(D.plan_waves(models, 1 << 50)) == 1
    with pytest.raises(D.DaliaError):
        D.plan_waves(models, max(per) // 2)


def test_mixed_refinement_batch_graph_single_bitwise(D):
    wl = W.scaled("mref", 8, 6, 3, 2, 60, seed=9)
    model = D.Model.from_workload(wl)
    rng = np.random.default_rng(4)
    th = wl.theta[None] + 0.05 * rng.standard_normal((3, wl.dim_theta))
    outs = {}
    for tag, kw, B in (("single", {}, 1), ("batch", {}, 3), ("graph", {"graph": True}, 3)):
        ws = D.Workspace([model] * B, mixed=True, **kw)
        res = []
        for _ in range(2):  # graph: capture, then a replay
            f, p, info = ws.fobj(th)
            torch.cuda.synchronize()
            res = (f.cpu().numpy().copy(), p.cpu().numpy().copy(), info.cpu().numpy().copy())
        outs[tag] = res
        del ws
    for tag in ("batch", "graph"):
        for a, b in zip(outs["single"], outs[tag]):
            assert np.array_equal(a, b), tag
    p = outs["single"][1]
    assert np.all(outs["single"][2] == 0)
    assert np.all(p[:, 7] <= 1e-12), p[:, 7]
