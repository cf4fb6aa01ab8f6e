"""Diagonal-block inverses formed inside the panel launches (DL_WS_FOLD_INV):
the left-looking inverse, one row of 64 x 64 tiles per panel step, instead
of the recursive GEMM inversion after each factorisation.  Every later step
(the [B; R] scaling, Schur updates, solve, selected inversion) consumes
these inverses, so the oracle's log-determinants, mean, marginal variances
and f_obj check them to the parity tolerances (FP64); the default path's
results agree to rounding.

Cases: blocks of 2, 3, 10 and 19 tiles (the inverse's first row, the
hand-over of G(j, j-1) through the accumulators, several rows), one- and
two-sided order, Q_p in a ring and stored in full, mixed precision, a batch
against single evaluations (bit for bit), graph replay, and the production
workloads against the stored banded-oracle values.
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
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_06938_amd import dalia
    dalia.lib()
    return dalia


CASES = {
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
    return (f.cpu().numpy(), parts.cpu().numpy(), info.cpu().numpy(),
            mu.cpu().numpy(), var.cpu().numpy())


@pytest.mark.parametrize("two_sided,keep_qp", [(False, False), (True, False), (True, True)])
@pytest.mark.parametrize("name", list(CASES))
def test_folded_inverse_against_oracle(D, name, two_sided, keep_qp):
    wl = CASES[name]()
    theta = wl.theta + 0.05 * np.sin(np.arange(wl.dim_theta) + 1.0)
    ref = oracle_ref(wl, theta)
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True, keep_qp=keep_qp, two_sided=two_sided,
                     fold_inverse=True)
    f, p, info, mu, var = evaluate(ws, theta)
    print(name, two_sided, keep_qp, f[0], ref["f"], flush=True)
    assert info.tolist() == [[0, 0]], name
    p = p[0]
    assert abs(p[1] - ref["logdet_p"]) <= 1e-10 * abs(ref["logdet_p"]), name
    assert abs(p[2] - ref["logdet_c"]) <= 1e-10 * abs(ref["logdet_c"]), name
    scale = abs(ref["logdet_p"]) + abs(ref["logdet_c"])
    assert abs(f[0] - ref["f"]) <= 1e-10 * scale, name
    assert np.max(np.abs(mu - ref["mu_bta"])) <= 1e-9 * np.max(np.abs(ref["mu_bta"]))
    np.testing.assert_allclose(var, ref["var_bta"], rtol=1e-9, err_msg=name)
    # the recursive inversion gives the same numbers up to rounding
    ws0 = D.Workspace(model, selinv=True, keep_qp=keep_qp, two_sided=two_sided)
    f0, p0, _, mu0, var0 = evaluate(ws0, theta)
    assert abs(p0[0][2] - p[2]) <= 1e-12 * abs(p[2])
    assert np.max(np.abs(mu0 - mu)) <= 1e-10 * np.max(np.abs(mu))
    np.testing.assert_allclose(var0, var, rtol=1e-10)


def test_folded_inverse_mixed_precision(D):
    wl = W.scaled("tri", 8, 5, 3, 2, 60, seed=4)
    model = D.Model.from_workload(wl)
    out = {}
    for tag, kw in (("fp64", {}), ("mixed", {"mixed": True})):
        ws = D.Workspace(model, selinv=True, two_sided=True, fold_inverse=True, **kw)
        out[tag] = evaluate(ws, wl.theta)
        del ws
    p64, pmx = out["fp64"][1][0], out["mixed"][1][0]
    assert out["mixed"][2].tolist() == [[0, 0]]
    assert pmx[7] <= 1e-12
    assert np.max(np.abs(out["mixed"][3] - out["fp64"][3])) <= \
        1e-9 * np.max(np.abs(out["fp64"][3]))
    assert abs(pmx[2] - p64[2]) <= 1e-4 * abs(p64[2])
    np.testing.assert_allclose(out["mixed"][4], out["fp64"][4], rtol=1e-2)


def test_folded_inverse_batch_equals_single_calls(D):
    wls = [W.scaled("u0", 13, 4, 1, 2, 48, seed=21),
           W.scaled("u1", 8, 7, 3, 1, 35, seed=22),
           W.scaled("u2", 7, 3, 1, 2, 30, seed=23)]
    models = [D.Model.from_workload(w) for w in wls]
    ws = D.Workspace(models, selinv=True, two_sided=True, fold_inverse=True)
    thetas = np.concatenate([w.theta for w in wls])
    fb, pb, ib = ws.fobj(thetas)
    var_b = ws.selinv().cpu().numpy()
    torch.cuda.synchronize()
    off = 0
    for k, (w, mdl) in enumerate(zip(wls, models)):
        ws1 = D.Workspace(mdl, selinv=True, two_sided=True, fold_inverse=True)
        f1, p1, i1 = ws1.fobj(w.theta)
        v1 = ws1.selinv().cpu().numpy()
        torch.cuda.synchronize()
        assert ib.cpu().numpy()[k].tolist() == [0, 0]
        assert fb.cpu().numpy()[k] == f1.cpu().numpy()[0], k
        assert np.array_equal(var_b[off:off + w.N], v1), k
        off += w.N


def test_folded_inverse_graph_replays_match_eager(D):
    wl = W.scaled("g", 12, 5, 1, 2, 100, seed=7)
    model = D.Model.from_workload(wl)
    eager = D.Workspace([model] * 2, two_sided=True, fold_inverse=True)
    graph = D.Workspace([model] * 2, two_sided=True, fold_inverse=True, graph=True)
    rng = np.random.default_rng(3)
    for r in range(4):
        th = wl.theta[None] + 0.05 * rng.standard_normal((2, wl.dim_theta))
        fg, pg, _ = graph.fobj(th)
        x = torch.randn(1000, device="cuda").sum()   # eager work in between
        torch.cuda.synchronize()
        fe, pe, _ = eager.fobj(th)
        torch.cuda.synchronize()
        assert np.array_equal(fg.cpu().numpy(), fe.cpu().numpy()), r
        assert np.array_equal(pg.cpu().numpy(), pe.cpu().numpy()), r
        del x


@pytest.mark.parametrize("name,make", [("c1", W.config1), ("c2", W.config2)])
def test_folded_inverse_fullsize_against_banded_oracle(D, name, make):
    path = os.path.join(GOLD, f"{name}_golden.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    g = json.load(open(path))
    wl = make()
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True, two_sided=True, fold_inverse=True)
    f, parts, info = ws.fobj(np.asarray(g["theta"]))
    mu = ws.mean()
    var = ws.selinv()
    torch.cuda.synchronize()
    p = parts.cpu().numpy()[0]
    assert info.cpu().tolist() == [[0, 0]]
    assert abs(p[1] - g["logdet_p"]) <= 1e-10 * abs(g["logdet_p"])
    assert abs(p[2] - g["logdet_c"]) <= 1e-10 * abs(g["logdet_c"])
    assert abs(p[0] - g["f"]) <= 1e-10 * (abs(g["logdet_p"]) + abs(g["logdet_c"]))
    mu_s = mu.cpu().numpy()[np.asarray(g["mu_index_bta"])]
    want = np.asarray(g["mu"])
    assert np.max(np.abs(mu_s - want)) <= 1e-9 * np.max(np.abs(want))
    v_s = var.cpu().numpy()[np.asarray(g["var_index_bta"])]
    np.testing.assert_allclose(v_s, np.asarray(g["var"]), rtol=1e-9)
