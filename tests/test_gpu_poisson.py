"""Poisson likelihood (non-Gaussian; Section II-A, conditional Gaussian distribution): the inner mode by damped
Newton on the GPU and f_obj by the Laplace approximation at it, against the
oracle's independent implementation (oracle/laplace.py) on the same seeded
count workloads.

The mode search over theta and the Hessian at its optimum run on the Poisson
f_obj as on the Gaussian one.

Tolerances (FP64): the mode is converged to ~1e-13 relative on both sides,
so the log-determinants and f_obj agree to 1e-10 of |log|Q_p|| + |log|Q_c||,
the mode to 1e-8 of its largest entry, and the marginal variances of the
Laplace approximation (diagonal of Q_c(x*)^{-1}) to 1e-8 relative.  The
Newton step counts may differ by one when a step ends within rounding of the
stopping threshold.  Batches equal single evaluations bit for bit (an
instance that has converged keeps its iterate).
"""
import numpy as np
import pytest

import workloads as W
from oracle import fobj as OF
from oracle import model as OM
from oracle.linalg import DenseSPD

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_06938_amd import dalia
    dalia.lib()
    return dalia


def _zeroed(wl):
    for r in wl.responses:
        r.y[:] = 0.0
    return wl


def _pois(name, nx, nt, nv, nr, m, seed, model="separable"):
    return lambda: W.scaled(name, nx, nt, nv, nr, m, seed=seed, model=model,
                            likelihood="poisson")


CASES = {
    "uni_2tiles": _pois("u", 10, 6, 1, 2, 300, 3),
    "tri_damped": _pois("t", 8, 5, 3, 2, 200, 3),          # first step halved
    "diff_uni": _pois("d", 13, 5, 1, 1, 90, 3, "diffusion"),
    "ragged_nt7": _pois("r", 9, 7, 1, 3, 140, 17),
    "uni_19tiles": _pois("s", 34, 4, 1, 2, 800, 18),        # b = 1156
    "tri_diff_nt6": _pois("td", 5, 6, 3, 2, 40, 15, "diffusion"),
    # degenerate cases: no observations (Q_c = Q_p, mode 0), all counts
    # zero, a single time step (one block), two responses
    "no_obs": _pois("e", 6, 3, 1, 2, 0, 1),
    "zero_counts": lambda: _zeroed(W.scaled("z", 6, 4, 1, 2, 120, seed=1,
                                            likelihood="poisson")),
    "nt1": _pois("n1", 8, 1, 1, 2, 100, 2),
    "bivariate": _pois("bv", 6, 5, 2, 1, 80, 2),
}


def oracle_ref(wl, theta):
    parts = OF.fobj_parts(wl, theta)
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


@pytest.mark.parametrize("variant", ["default", "two_sided_fold", "keep_qp"])
@pytest.mark.parametrize("name", list(CASES))
def test_poisson_laplace_against_oracle(D, name, variant):
    wl = CASES[name]()
    theta = wl.theta + 0.05 * np.sin(np.arange(wl.dim_theta) + 1.0)
    print(name, variant, flush=True)
    ref = oracle_ref(wl, theta)
    assert ref["converged"]
    model = D.Model.from_workload(wl)
    assert model.dim_theta == wl.dim_theta
    kw = dict(default={}, two_sided_fold=dict(two_sided=True, fold_inverse=True),
              keep_qp=dict(keep_qp=True))[variant]
    ws = D.Workspace(model, selinv=True, **kw)
    f, p, info, mu, var = evaluate(ws, theta)
    steps = ws.newton_steps()
    p = p[0]
    print(f"  f {f[0]:.12f} oracle {ref['f']:.12f}  steps {steps[0]} oracle "
          f"{ref['newton_steps']}  rel residual {p[7]:.2e}", flush=True)
    assert info.tolist() == [[0, 0]]
    assert abs(int(steps[0]) - ref["newton_steps"]) <= 1
    scale = abs(ref["logdet_p"]) + abs(ref["logdet_c"])
    assert abs(p[1] - ref["logdet_p"]) <= 1e-10 * abs(ref["logdet_p"])
    assert abs(p[2] - ref["logdet_c"]) <= 1e-10 * scale
    assert abs(f[0] - ref["f"]) <= 1e-10 * scale
    assert abs(p[4] - ref["quad_obs"]) <= 1e-10 * scale
    assert p[6] == 0.0                       # no Gaussian constant
    assert p[7] <= 1e-9                      # gradient of h at the mode
    assert np.max(np.abs(mu - ref["mu_bta"])) <= 1e-8 * np.max(np.abs(ref["mu_bta"]))
    np.testing.assert_allclose(var, ref["var_bta"], rtol=1e-8)


def test_poisson_batch_equals_single_calls(D):
    wls = [CASES["uni_2tiles"](), CASES["tri_damped"](), CASES["diff_uni"]()]
    models = [D.Model.from_workload(w) for w in wls]
    ws = D.Workspace(models, selinv=True)
    thetas = np.concatenate([w.theta for w in wls])
    fb, pb, ib = ws.fobj(thetas)
    var_b = ws.selinv().cpu().numpy()
    steps_b = ws.newton_steps()
    torch.cuda.synchronize()
    off = 0
    for k, (w, mdl) in enumerate(zip(wls, models)):
        ws1 = D.Workspace(mdl, selinv=True)
        f1, p1, i1 = ws1.fobj(w.theta)
        v1 = ws1.selinv().cpu().numpy()
        torch.cuda.synchronize()
        assert ws1.newton_steps()[0] == steps_b[k] > 0
        assert fb.cpu().numpy()[k] == f1.cpu().numpy()[0], k
        assert np.array_equal(pb.cpu().numpy()[k], p1.cpu().numpy()[0]), k
        assert np.array_equal(var_b[off:off + w.N], v1), k
        off += w.N


def test_poisson_several_passes_and_graph_flag(D):
    """ntheta > B on one model (two passes, the second one partly idle), and
    a DL_WS_GRAPH workspace (the mode search runs eagerly): both equal
    single evaluations bit for bit."""
    wl = CASES["uni_2tiles"]()
    model = D.Model.from_workload(wl)
    rng = np.random.default_rng(5)
    th = wl.theta[None] + 0.1 * rng.standard_normal((3, wl.dim_theta))
    ws2 = D.Workspace([model] * 2)
    f2, p2, _ = ws2.fobj(th)
    wsg = D.Workspace(model, graph=True)
    single = []
    for r in range(3):
        f1, _, _ = wsg.fobj(th[r])
        single.append(f1.cpu().numpy()[0])
    torch.cuda.synchronize()
    assert f2.cpu().numpy().tolist() == single
    ref = [OF.fobj(wl, t) for t in th]
    np.testing.assert_allclose(single, ref, rtol=1e-11)


def test_poisson_fobj_selinv_equals_fobj_then_selinv(D):
    wl = CASES["tri_damped"]()
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True, two_sided=True)
    f, p, i, var = ws.fobj_selinv(wl.theta)
    var = var.cpu().numpy()
    ws2 = D.Workspace(model, selinv=True, two_sided=True)
    f2, p2, _ = ws2.fobj(wl.theta)
    var2 = ws2.selinv().cpu().numpy()
    torch.cuda.synchronize()
    assert f.cpu().numpy().tolist() == f2.cpu().numpy().tolist()
    assert np.array_equal(var, var2)


def test_poisson_rejects_mixed_likelihoods(D):
    pw = CASES["uni_2tiles"]()
    gw = W.config0()
    pm, gm = D.Model.from_workload(pw), D.Model.from_workload(gw)
    with pytest.raises(D.DaliaError):
        D.Workspace([pm, gm])
    # a Gaussian workspace reports no Newton steps
    ws = D.Workspace(gm)
    ws.fobj(gw.theta)
    torch.cuda.synchronize()
    assert ws.newton_steps().tolist() == [0]


def test_poisson_production_size_converges(D):
    """Counts on the production univariate mesh (45 x 45, nt = 100,
    m = 200000): the mode search converges, the gradient at the mode is
    at rounding level, and the two-sided order with folded inverses agrees
    with the default order to rounding."""
    wl = W.make_univariate("c1_poisson", 45, 100, 4, 200_000, seed=0,
                           likelihood="poisson")
    model = D.Model.from_workload(wl)
    out = {}
    for tag, kw in (("default", {}), ("two_fold", dict(two_sided=True, fold_inverse=True))):
        ws = D.Workspace(model, **kw)
        f, p, info = ws.fobj(wl.theta)
        torch.cuda.synchronize()
        out[tag] = (f.cpu().numpy()[0], p.cpu().numpy()[0], ws.newton_steps()[0])
        print(tag, out[tag][0], "steps", out[tag][2], "rel residual", out[tag][1][7], flush=True)
        assert info.cpu().tolist() == [[0, 0]]
        del ws
    (f0, p0, s0), (f1, p1, s1) = out["default"], out["two_fold"]
    assert np.isfinite(f0) and 0 < s0 <= 20 and abs(s1 - s0) <= 1
    assert p0[7] <= 1e-9 and p1[7] <= 1e-9
    assert abs(f1 - f0) <= 1e-10 * (abs(p0[1]) + abs(p0[2]))


def test_poisson_mode_search_and_hessian_match_oracle(D):
    """The hyperparameter mode search (Eq. 9, batched central differences,
    Eq. 10) and the Hessian at the mode on the Poisson f_obj: the GPU
    drivers reach the oracle BFGS optimum value (|F - F*| <= 1e-6 |F*|), and
    the second differences at the oracle's optimum agree with the oracle's
    (|dH| <= 2e-12 |f| / h^2, as for the Gaussian likelihood)."""
    from oracle import bfgs as OB
    from oracle import hessian as OH
    from paper_2507_06938_amd import hessian as GH
    from paper_2507_06938_amd import optimize as O
    wl = W.scaled("opt_pois", 5, 4, 1, 2, 60, seed=11, likelihood="poisson")
    theta0 = W.random_theta_near(wl.theta, 0.25, seed=3)
    F = lambda t: -OF.fobj(wl, t)
    fg = lambda t: (F(t), OB.central_gradient(F, t, 1e-3))
    xs, fs, _ = OB.bfgs_minimize(fg, theta0, max_iter=300, ftol=1e-13, gtol=1e-6)
    model = D.Model.from_workload(wl)
    ev = O.Evaluator(model, batch=2 * wl.dim_theta + 1)
    tr = O.fd_bfgs(ev, theta0, h=1e-3, ftol=1e-13, gtol=1e-6, max_iter=300)
    print(f"oracle F*={fs:.12f}  gpu F={tr.f[-1]:.12f}  iters={len(tr.f) - 1}", flush=True)
    assert abs(tr.f[-1] - fs) <= 1e-6 * abs(fs)
    # the evaluator warm-starts the inner search by default for counts, and a
    # cold evaluator reaches the same optimum
    assert ev.ws.newton_steps().max() <= 4
    ev_cold = O.Evaluator(model, batch=2 * wl.dim_theta + 1, warm_start=False)
    tr_cold = O.fd_bfgs(ev_cold, theta0, h=1e-3, ftol=1e-13, gtol=1e-6, max_iter=300)
    assert abs(tr_cold.f[-1] - fs) <= 1e-6 * abs(fs)
    d = wl.dim_theta
    ws = D.Workspace([model] * (2 * d * d + 1))
    H_gpu, f0, vals = GH.fobj_hessian(ws, xs, 1e-3)
    ref_vals = np.array([OF.fobj(wl, p) for p in OH.hessian_stencil(xs, 1e-3)])
    H_ref = OH.hessian_from_values(ref_vals, d, 1e-3)
    print("max |dH|", np.max(np.abs(H_gpu - H_ref)), flush=True)
    assert np.max(np.abs(H_gpu - H_ref)) <= 2e-12 * abs(ref_vals[0]) / 1e-6
    assert np.linalg.eigvalsh(H_gpu).max() < 0
    np.testing.assert_allclose(GH.marginal_sd(H_gpu), OH.gaussian_marginal_sd(H_ref), rtol=1e-5)


def test_poisson_warm_start(D):
    """DL_WS_WARM_START: the first pass starts from x = 0 (identical to a
    cold workspace), later passes from the previous mode; at a nearby theta
    the search takes fewer steps and reaches the same f_obj to rounding."""
    wl = CASES["uni_19tiles"]()
    model = D.Model.from_workload(wl)
    warm = D.Workspace(model, warm_start=True)
    cold = D.Workspace(model)
    th1 = wl.theta
    th2 = wl.theta + 0.02 * np.array([1.0, -1.0, 0.5])
    fw1, _, _ = warm.fobj(th1)
    fc1, _, _ = cold.fobj(th1)
    torch.cuda.synchronize()
    assert fw1.cpu().tolist() == fc1.cpu().tolist()
    assert warm.newton_steps().tolist() == cold.newton_steps().tolist()
    fw2, pw2, _ = warm.fobj(th2)
    sw = int(warm.newton_steps()[0])
    fc2, pc2, _ = cold.fobj(th2)
    sc = int(cold.newton_steps()[0])
    torch.cuda.synchronize()
    print("steps warm", sw, "cold", sc, flush=True)
    assert 0 < sw < sc
    p = pc2.cpu().numpy()[0]
    scale = abs(p[1]) + abs(p[2])
    assert abs(fw2.item() - fc2.item()) <= 1e-10 * scale
    assert abs(fw2.item() - OF.fobj(wl, th2)) <= 1e-10 * scale
    assert pw2.cpu().numpy()[0][7] <= 1e-9


@pytest.mark.parametrize("kw", [{}, {"two_sided": True, "fold_inverse": True}])
@pytest.mark.parametrize("name,make", [
    ("c1_poisson", lambda: W.config1(likelihood="poisson")),
    ("c2_poisson", lambda: W.config2(likelihood="poisson"))])
def test_poisson_fullsize_against_banded_oracle(D, name, make, kw):
    """The production-size count workloads (univariate 45 x 45, nt = 100,
    m = 200000; trivariate 30 x 30, nt = 48, m = 3 x 43200) against values
    stored by tests/golden/make_golden.py (oracle: damped Newton with RCM +
    banded LAPACK Cholesky): log-determinants, f_obj, the inner mode and the
    Laplace marginal variances at seeded positions."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", f"{name}_golden.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    g = json.load(open(path))
    wl = make()
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True, **kw)
    f, parts, info = ws.fobj(np.asarray(g["theta"]))
    mu = ws.mean()
    var = ws.selinv()
    torch.cuda.synchronize()
    p = parts.cpu().numpy()[0]
    steps = int(ws.newton_steps()[0])
    print(kw, "f", p[0], "oracle", g["f"], "steps", steps, "oracle", g["newton_steps"], flush=True)
    assert info.cpu().tolist() == [[0, 0]]
    assert abs(steps - g["newton_steps"]) <= 1
    assert abs(p[1] - g["logdet_p"]) <= 1e-10 * abs(g["logdet_p"])
    scale = abs(g["logdet_p"]) + abs(g["logdet_c"])
    assert abs(p[2] - g["logdet_c"]) <= 1e-10 * scale
    assert abs(p[0] - g["f"]) <= 1e-10 * scale
    mu_s = mu.cpu().numpy()[np.asarray(g["mu_index_bta"])]
    want = np.asarray(g["mu"])
    assert np.max(np.abs(mu_s - want)) <= 1e-8 * np.max(np.abs(want))
    v_s = var.cpu().numpy()[np.asarray(g["var_index_bta"])]
    np.testing.assert_allclose(v_s, np.asarray(g["var"]), rtol=1e-8)
    v = var.cpu().numpy()
    assert np.all(np.isfinite(v)) and np.all(v > 0)


def test_poisson_without_observations_is_the_prior(D):
    """No observations: Q_c = Q_p, the mode is 0 after one Newton step, and
    f_obj reduces to log p(theta) (the two half log-determinants cancel)."""
    wl = CASES["no_obs"]()
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True)
    f, p, info = ws.fobj(wl.theta)
    mu = ws.mean()
    torch.cuda.synchronize()
    p = p.cpu().numpy()[0]
    assert info.cpu().tolist() == [[0, 0]] and ws.newton_steps().tolist() == [1]
    assert not np.any(mu.cpu().numpy())
    assert p[2] == p[1] and p[3] == 0.0 and p[4] == 0.0
    assert f.item() == pytest.approx(OM.log_prior_theta(wl.theta, wl.theta_prior_mean,
                                                        wl.theta_prior_sd), rel=1e-14)


def test_poisson_low_level_entry_points_use_the_last_iterate(D):
    """After f_obj, bta_assemble and bta_factor of Q_c build Q_c with the
    weights of the inner mode (the header's documented behaviour), so they
    reproduce log|Q_c(x*)| bit for bit, and bta_solve of the assembled
    right-hand side A^T (g + D A x*) returns x* itself (one more Newton
    step from the mode)."""
    wl = CASES["uni_2tiles"]()
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model)
    f, parts, _ = ws.fobj(wl.theta)
    mode = ws.mean().clone()
    torch.cuda.synchronize()
    ws.assemble(wl.theta, D.DL_QC)
    ld, info = ws.factor(D.DL_QC)
    ws.solve()
    x = ws.mean()
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0]
    assert ld.cpu().item() == parts.cpu().numpy()[0][2]
    m = mode.cpu().numpy()
    assert np.max(np.abs(x.cpu().numpy() - m)) <= 1e-11 * np.max(np.abs(m))


@pytest.mark.parametrize("name", ["uni_19tiles", "tri_damped"])
def test_poisson_mixed_precision(D, name):
    """DL_WS_MIXED with counts: the Newton solves are refined in FP64, so the
    mode and the step count match the FP64 workspace; log|Q_p| and log|Q_c|
    carry the FP32 error of the off-diagonal blocks (1e-4 relative, as for
    the Gaussian likelihood) and the variances agree to 1e-2."""
    wl = CASES[name]()
    model = D.Model.from_workload(wl)
    out = {}
    for tag, kw in (("fp64", {}), ("mixed", {"mixed": True})):
        ws = D.Workspace(model, selinv=True, two_sided=True, **kw)
        out[tag] = evaluate(ws, wl.theta) + (ws.newton_steps()[0],)
        del ws
    f64, p64, i64, mu64, v64, s64 = out["fp64"]
    fmx, pmx, imx, mumx, vmx, smx = out["mixed"]
    print(name, "steps", s64, smx, "f", f64[0], fmx[0], flush=True)
    assert imx.tolist() == [[0, 0]] and abs(int(smx) - int(s64)) <= 1
    assert np.max(np.abs(mumx - mu64)) <= 1e-9 * np.max(np.abs(mu64))
    assert pmx[0][7] <= 1e-12
    assert abs(pmx[0][1] - p64[0][1]) <= 1e-4 * abs(p64[0][1])
    assert abs(pmx[0][2] - p64[0][2]) <= 1e-4 * abs(p64[0][2])
    assert abs(fmx[0] - f64[0]) <= 1e-4 * abs(p64[0][2])
    np.testing.assert_allclose(vmx, v64, rtol=1e-2)
