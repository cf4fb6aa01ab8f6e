"""The call the benchmark times -- fobj_selinv_eval on a workspace in the
two-sided elimination order with the diagonal blocks' inverses formed inside
the panel launches, GEMM tiles from the autotuner's cache -- checked against
the oracle:

  * small cases: bit for bit against fobj_eval followed by bta_selinv on the
    same workspace (the launches and inputs are the same), and against the
    oracle's dense evaluation (log-determinants, f_obj, mean, every marginal
    variance) to the parity tolerances; two calls in a row with different
    thetas;
  * production sizes (c1: 45x45 mesh, n_t = 100; c2: trivariate 30x30 mesh,
    n_t = 48): against the values stored by tests/golden/make_golden.py (RCM
    + banded LAPACK Cholesky): f_obj and every part, the mean at the stored
    positions and the marginal variances at the stored positions.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import fobj as OF
from oracle import model as OM
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


SMALL = {
    "c0": W.config0,
    "uni_nt9_ragged": lambda: W.scaled("t9", 9, 9, 1, 3, 150, seed=21),
    "tri_nt6": lambda: W.scaled("t6", 6, 6, 3, 2, 50, seed=22),
    "uni_b192_nt5": lambda: W.scaled("t5", 14, 5, 1, 2, 300, seed=23),
    "diff_nt6": lambda: W.scaled("td", 7, 6, 1, 2, 90, seed=24, model="diffusion"),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_timed_configuration_small(D, name):
    wl = SMALL[name]()
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True, two_sided=True, fold_inverse=True)
    ws.autotune(TILES)
    perm = OM.bta_permutation(wl.nv, wl.ns, wl.nt, wl.nr)
    rng = np.random.default_rng(5)
    for call in range(2):
        theta = wl.theta + 0.05 * rng.standard_normal(wl.dim_theta)
        print(f"{name} call {call} N={wl.N}", flush=True)
        f1, p1, i1, v1 = ws.fobj_selinv(theta)
        torch.cuda.synchronize()
        mu1 = ws.mean()
        torch.cuda.synchronize()
        r1 = [x.cpu().numpy().copy() for x in (f1, p1, i1, v1, mu1)]
        f0, p0, i0 = ws.fobj(theta)
        v0 = ws.selinv()
        mu0 = ws.mean()
        torch.cuda.synchronize()
        for a, b in zip(r1, (f0, p0, i0, v0, mu0)):
            assert np.array_equal(a, b.cpu().numpy()), (name, call)
        ref = OF.fobj_parts(wl, theta, return_factors=True)
        p = r1[1][0]
        assert r1[2].tolist() == [[0, 0]]
        assert abs(p[1] - ref["logdet_p"]) <= 1e-10 * abs(ref["logdet_p"])
        assert abs(p[2] - ref["logdet_c"]) <= 1e-10 * abs(ref["logdet_c"])
        scale = abs(ref["logdet_p"]) + abs(ref["logdet_c"])
        assert abs(p[0] - ref["f"]) <= 1e-10 * scale
        assert abs(p[5] - ref["log_prior"]) <= 1e-12 * max(1.0, abs(ref["log_prior"]))
        mu_ref = ref["mu"][perm]
        assert np.max(np.abs(r1[4] - mu_ref)) <= 1e-9 * np.max(np.abs(mu_ref))
        var_ref = DenseSPD(ref["Qc"]).inv_diag()[perm]
        np.testing.assert_allclose(r1[3], var_ref, rtol=1e-9)


@pytest.mark.parametrize("name,make", [("c1", W.config1), ("c2", W.config2)])
def test_timed_call_at_production_size(D, name, make):
    g = json.load(open(os.path.join(GOLD, f"{name}_golden.json")))
    wl = make()
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True, two_sided=True, fold_inverse=True)
    ws.autotune(TILES)
    theta = np.asarray(g["theta"])
    print(f"{name} N={wl.N}", flush=True)
    f, parts, info, var = ws.fobj_selinv(theta)
    torch.cuda.synchronize()
    mu = ws.mean()
    torch.cuda.synchronize()
    p = parts.cpu().numpy()[0]
    assert info.cpu().tolist() == [[0, 0]]
    assert abs(p[1] - g["logdet_p"]) <= 1e-10 * abs(g["logdet_p"])
    assert abs(p[2] - g["logdet_c"]) <= 1e-10 * abs(g["logdet_c"])
    scale = abs(g["logdet_p"]) + abs(g["logdet_c"])
    assert abs(p[0] - g["f"]) <= 1e-10 * scale
    assert abs(f.item() - p[0]) == 0.0
    for k, key in ((3, "quad_p"), (4, "quad_obs")):
        assert abs(p[k] - g[key]) <= 1e-9 * abs(g[key]), key
    assert abs(p[5] - g["log_prior"]) <= 1e-12 * max(1.0, abs(g["log_prior"]))
    mu_s = mu.cpu().numpy()[np.asarray(g["mu_index_bta"])]
    want = np.asarray(g["mu"])
    assert np.max(np.abs(mu_s - want)) <= 1e-9 * np.max(np.abs(want))
    v = var.cpu().numpy()
    np.testing.assert_allclose(v[np.asarray(g["var_index_bta"])], np.asarray(g["var"]),
                               rtol=1e-9)
    assert np.all(np.isfinite(v)) and np.all(v > 0)
