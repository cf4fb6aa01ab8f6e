"""Diagonal blocks factored by one persistent launch per elimination step
(DL_WS_DAG): workgroups take 64 x 64 tile tasks -- tile factor, panel solve,
trailing update, inverse accumulation and inverse row -- from a fixed list
and wait on per-tile readiness counters (the list itself is checked on the
CPU by tests/test_dag_schedule.py).  Every later step (the [B; R] scaling,
Schur updates, solve, selected inversion) consumes the resulting inverses,
so the oracle's log-determinants, mean, marginal variances and f_obj check
them to the parity tolerances (FP64).

Cases: blocks of 1, 2, 3, 10 and 19 tiles, one- and two-sided order, Q_p in
a ring and stored in full, mixed precision, repeated calls (the launch
resets its counters itself), a batch against single evaluations, graph
replay, a planted non-positive pivot, and the production workloads in the
benchmark's configuration against the stored banded-oracle values.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import model as OM
from oracle import fobj as OF
from oracle.linalg import DenseSPD

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")
TILES = os.path.join(ROOT, "paper_2507_06938_amd", "tiles_gfx950.txt")


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_06938_amd import dalia
    dalia.lib()
    return dalia


CASES = {
    "one_tile": lambda: W.scaled("t1", 6, 5, 1, 2, 60, seed=3),           # b = 36
    "c0_2tiles": lambda: W.config0(),                                    # b = 100
    "tri_3tiles": lambda: W.scaled("tri", 8, 5, 3, 2, 60, seed=4),      # b = 192
    "uni_10tiles": lambda: W.scaled("u10", 25, 4, 1, 2, 300, seed=19),  # b = 625
    "uni_19tiles": lambda: W.scaled("sp", 34, 4, 1, 2, 800, seed=18),   # b = 1156
    "diff_3tiles": lambda: W.scaled("dt", 13, 5, 1, 1, 90, seed=20, model="diffusion"),
}


def oracle_ref(wl, theta):
    parts = OF.fobj_parts(wl, theta, return_factors=True)
    perm = OM.bta_permutation(wl.nv, wl.ns, wl.nt, wl.nr)
    parts["mu_bta"] = parts["mu"][perm]
    parts["var_bta"] = DenseSPD(parts["Qc"]).inv_diag()[perm]
    return parts


def evaluate(ws, theta):
    f, parts, info = ws.fobj(theta)
    mu = ws.mean()
    var = ws.selinv()
    torch.cuda.synchronize()
    return (f.cpu().numpy(), parts.cpu().numpy(), info.cpu().numpy(), mu.cpu().numpy(),
            var.cpu().numpy())


def check_against(ref, out, name):
    f, p, info, mu, var = out
    assert info.tolist() == [[0, 0]], name
    p = p[0]
    assert abs(p[1] - ref["logdet_p"]) <= 1e-10 * abs(ref["logdet_p"]), name
    assert abs(p[2] - ref["logdet_c"]) <= 1e-10 * abs(ref["logdet_c"]), name
    scale = abs(ref["logdet_p"]) + abs(ref["logdet_c"])
    assert abs(p[0] - ref["f"]) <= 1e-10 * scale, name
    assert np.max(np.abs(mu - ref["mu_bta"])) <= 1e-9 * np.max(np.abs(ref["mu_bta"])), name
    np.testing.assert_allclose(var, ref["var_bta"], rtol=1e-9, err_msg=name)


@pytest.mark.parametrize("two_sided,keep_qp", [(False, False), (True, False), (True, True)])
@pytest.mark.parametrize("name", list(CASES))
def test_dag_against_oracle(D, name, two_sided, keep_qp):
    wl = CASES[name]()
    theta = wl.theta + 0.05 * np.sin(np.arange(wl.dim_theta) + 2.0)
    print(f"{name} two_sided={two_sided} keep_qp={keep_qp} b={wl.b}", flush=True)
    ref = oracle_ref(wl, theta)
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True, dag=True, two_sided=two_sided, keep_qp=keep_qp)
    out = evaluate(ws, theta)
    check_against(ref, out, name)
    # again: the launches reset their counters themselves; bit for bit
    out2 = evaluate(ws, theta)
    for a, b in zip(out, out2):
        assert np.array_equal(a, b), name


def test_dag_matches_panel_path_to_rounding(D):
    wl = CASES["uni_19tiles"]()
    model = D.Model.from_workload(wl)
    outs = {}
    for tag, kw in (("panel", {"fold_inverse": True}), ("dag", {"dag": True})):
        ws = D.Workspace(model, selinv=True, two_sided=True, **kw)
        outs[tag] = evaluate(ws, wl.theta)
        del ws
    pp, pd = outs["panel"][1][0], outs["dag"][1][0]
    assert abs(pp[2] - pd[2]) <= 1e-12 * abs(pp[2])
    np.testing.assert_allclose(outs["dag"][4], outs["panel"][4], rtol=1e-11)


def test_dag_mixed_precision(D):
    wl = CASES["tri_3tiles"]()
    model = D.Model.from_workload(wl)
    ref = oracle_ref(wl, wl.theta)
    ws = D.Workspace(model, selinv=True, dag=True, mixed=True, two_sided=True)
    f, p, info, mu, var = evaluate(ws, wl.theta)
    assert info.tolist() == [[0, 0]]
    assert abs(p[0][2] - ref["logdet_c"]) <= 1e-4 * abs(ref["logdet_c"])
    assert p[0][7] <= 1e-12
    assert np.max(np.abs(mu - ref["mu_bta"])) <= 1e-9 * np.max(np.abs(ref["mu_bta"]))


def test_dag_batch_and_graph_equal_single(D):
    wls = [CASES["c0_2tiles"](), CASES["tri_3tiles"](), CASES["uni_10tiles"]()]
    models = [D.Model.from_workload(w) for w in wls]
    th = np.concatenate([w.theta for w in wls])
    single = []
    for m, w in zip(models, wls):
        ws = D.Workspace(m, dag=True)
        f, p, info = ws.fobj(w.theta)
        torch.cuda.synchronize()
        single.append((f.cpu().numpy()[0], p.cpu().numpy()[0].copy()))
        del ws
    for graph in (False, True):
        ws = D.Workspace(models, dag=True, graph=graph)
        for rep in range(2):
            f, p, info = ws.fobj(th)
            torch.cuda.synchronize()
            assert np.all(info.cpu().numpy() == 0)
            for k in range(len(wls)):
                assert f.cpu().numpy()[k] == single[k][0], (graph, rep, k)
                assert np.array_equal(p.cpu().numpy()[k], single[k][1]), (graph, rep, k)
        del ws


@pytest.mark.parametrize("two_sided", [False, True])
def test_dag_planted_bad_pivot(D, two_sided):
    wl = W.scaled("pivot", 9, 7, 1, 3, 140, seed=17)  # b = 81, nt = 7
    model = D.Model.from_workload(wl)
    b = wl.b
    ws = D.Workspace(model, selinv=True, dag=True, two_sided=two_sided)
    for t, r in ((0, 0), (2, 70), ((wl.nt + 1) // 2, 64), (wl.nt - 1, 5)):
        ws.assemble(wl.theta, D.DL_QC)
        Dt = ws.get_block(D.DL_QC, 0, t).cpu().numpy().copy()
        Dt[r, r] = -1.0
        ws.set_block(D.DL_QC, 0, t, torch.tensor(Dt, dtype=torch.float64, device="cuda"))
        ld, info = ws.factor(D.DL_QC)
        torch.cuda.synchronize()
        print(f"two_sided={two_sided} t={t} r={r} info={info.item()}", flush=True)
        assert info.item() == t * b + r + 1
    # a healthy evaluation afterwards (the aborted tiles left no state behind)
    ref = oracle_ref(wl, wl.theta)
    ws2 = D.Workspace(model, selinv=True, dag=True, two_sided=two_sided)
    check_against(ref, evaluate(ws2, wl.theta), "after")
    check_against(ref, evaluate(ws, wl.theta), "same workspace after")


@pytest.mark.parametrize("name,make", [("c1", W.config1), ("c2", W.config2)])
def test_dag_production_size_timed_configuration(D, name, make):
    g = json.load(open(os.path.join(GOLD, f"{name}_golden.json")))
    wl = make()
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True, two_sided=True, dag=True)
    ws.autotune(TILES)
    print(f"{name} N={wl.N}", flush=True)
    f, parts, info, var = ws.fobj_selinv(np.asarray(g["theta"]))
    torch.cuda.synchronize()
    mu = ws.mean().cpu().numpy()
    p = parts.cpu().numpy()[0]
    assert info.cpu().tolist() == [[0, 0]]
    assert abs(p[1] - g["logdet_p"]) <= 1e-10 * abs(g["logdet_p"])
    assert abs(p[2] - g["logdet_c"]) <= 1e-10 * abs(g["logdet_c"])
    assert abs(p[0] - g["f"]) <= 1e-10 * (abs(g["logdet_p"]) + abs(g["logdet_c"]))
    want = np.asarray(g["mu"])
    assert np.max(np.abs(mu[np.asarray(g["mu_index_bta"])] - want)) <= 1e-9 * np.max(np.abs(want))
    v = var.cpu().numpy()
    np.testing.assert_allclose(v[np.asarray(g["var_index_bta"])], np.asarray(g["var"]), rtol=1e-9)
