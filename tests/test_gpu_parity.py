"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by
element, on seeded workloads small enough for the dense oracle but spanning
several 64x64 tiles, ragged block sizes and the degenerate cases (one time
step, no fixed effects), for the separable and the non-separable
(diffusion-based) model families.

Tolerances (FP64 throughout, condition numbers <= ~1e5 at these sizes):
  log-determinants   relative 1e-10
  mean mu            1e-9 * max|mu|
  diag(Q_c^-1)       relative 1e-9
  f_obj              absolute 1e-10 * (|log|Q_p|| + |log|Q_c||)
  assembled blocks   1e-12 * max|block| (same sums, different order)
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import model as OM
from oracle import fobj as OF
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


def oracle_case(wl, theta):
    parts = OF.fobj_parts(wl, theta, return_factors=True)
    perm = OM.bta_permutation(wl.nv, wl.ns, wl.nt, wl.nr)
    parts["perm"] = perm
    parts["Qp_bta"] = parts["Qp"][perm][:, perm].toarray()
    parts["Qc_bta"] = parts["Qc"][perm][:, perm].toarray()
    parts["mu_bta"] = parts["mu"][perm]
    parts["r_bta"] = parts["r"][perm]
    parts["var_bta"] = DenseSPD(parts["Qc"]).inv_diag()[perm]
    return parts


CASES = {
    "c0": lambda: W.config0(),
    "tri_small": lambda: W.scaled("tri", 5, 4, 3, 2, 40, seed=4),
    "ragged_b81": lambda: W.scaled("rag", 9, 3, 1, 3, 120, seed=7),
    "b64_exact": lambda: W.scaled("b64", 8, 5, 1, 1, 80, seed=8),
    "one_step": lambda: W.scaled("one", 7, 1, 1, 2, 50, seed=9),
    "no_fixed": lambda: W.scaled("nof", 6, 4, 1, 0, 60, seed=10),
    "bivariate": lambda: W.scaled("bi", 6, 3, 2, 1, 40, seed=11),
    "multi_tile": lambda: W.scaled("mt", 12, 3, 1, 2, 300, seed=12),
    # b = 1156: 19 tiles per block, so the first panels of every diagonal
    # block are solved in place before their trailing update
    "solved_panels": lambda: W.scaled("sp", 34, 4, 1, 2, 800, seed=18),
    # non-separable diffusion-based model: 25-point spatial stencil, the
    # fourth FEM piece, nt = 2 (both steps are end steps) and ragged tiles
    "diff_uni": lambda: W.scaled("du", 7, 5, 1, 2, 80, seed=13, model="diffusion"),
    "diff_two_steps": lambda: W.scaled("d2", 6, 2, 1, 1, 40, seed=14,
                                       model="diffusion"),
    "diff_tri": lambda: W.scaled("dt", 5, 4, 3, 2, 40, seed=15, model="diffusion"),
    "diff_multi_tile": lambda: W.scaled("dm", 11, 3, 1, 2, 250, seed=16,
                                        model="diffusion"),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, D):
    wl = CASES[request.param]()
    theta = wl.theta + 0.05 * np.sin(np.arange(wl.dim_theta) + 1.0)
    ref = oracle_case(wl, theta)
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True, keep_qp=True)
    return request.param, wl, theta, ref, model, ws


def _close(got, want, rel, what):
    err = np.max(np.abs(got - want)) if np.size(want) else 0.0
    scale = max(np.max(np.abs(want)) if np.size(want) else 0.0, 1e-300)
    assert err <= rel * scale, f"{what}: max abs err {err:.3e} vs scale {scale:.3e}"


def test_assembled_blocks(D, case):
    name, wl, theta, ref, model, ws = case
    ws.assemble(theta, D.DL_BOTH)
    torch.cuda.synchronize()
    b, nt, a = wl.b, wl.nt, wl.a
    for which, Q in ((D.DL_QP, ref["Qp_bta"]), (D.DL_QC, ref["Qc_bta"])):
        for t in range(nt):
            sl = slice(t * b, (t + 1) * b)
            Dt = ws.get_block(which, 0, t).cpu().numpy()
            _close(Dt, np.tril(Q[sl, sl]), 1e-12, f"{name} D_{t}")
            if t + 1 < nt:
                sl2 = slice((t + 1) * b, (t + 2) * b)
                Bt = ws.get_block(which, 1, t).cpu().numpy()
                _close(Bt, Q[sl2, sl], 1e-12, f"{name} B_{t}")
            if which == D.DL_QC and a > 0:
                Rt = ws.get_block(which, 2, t).cpu().numpy()
                _close(Rt, Q[nt * b:, sl], 1e-12, f"{name} R_{t}")
        if a > 0:
            P = ws.get_block(which, 3).cpu().numpy()
            _close(P, np.tril(Q[nt * b:, nt * b:]), 1e-12, f"{name} tip")
    rhs = ws.get_block(D.DL_QC, 4).cpu().numpy()
    _close(rhs, ref["r_bta"], 1e-12, f"{name} rhs")


def test_logdets_mean_variances(D, case):
    name, wl, theta, ref, model, ws = case
    ws.assemble(theta, D.DL_BOTH)
    ld, info = ws.factor(D.DL_BOTH)
    mu = ws.solve()
    var = ws.selinv()
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, 0]
    ldp, ldc = ld.cpu().tolist()
    assert abs(ldp - ref["logdet_p"]) <= 1e-10 * abs(ref["logdet_p"]), name
    assert abs(ldc - ref["logdet_c"]) <= 1e-10 * abs(ref["logdet_c"]), name
    _close(mu.cpu().numpy(), ref["mu_bta"], 1e-9, f"{name} mu")
    v = var.cpu().numpy()
    np.testing.assert_allclose(v, ref["var_bta"], rtol=1e-9, err_msg=name)


def test_fobj_and_parts(D, case):
    name, wl, theta, ref, model, ws = case
    f, parts, info = ws.fobj(theta)
    torch.cuda.synchronize()
    p = parts.cpu().numpy()[0]
    scale = abs(ref["logdet_p"]) + abs(ref["logdet_c"])
    assert info.cpu().tolist() == [[0, 0]]
    assert abs(f.item() - ref["f"]) <= 1e-10 * scale, (name, f.item(), ref["f"])
    assert abs(p[0] - ref["f"]) <= 1e-10 * scale
    assert abs(p[3] - ref["quad_p"]) <= 1e-9 * max(1.0, abs(ref["quad_p"]))
    assert abs(p[4] - ref["quad_obs"]) <= 1e-9 * max(1.0, abs(ref["quad_obs"]))
    assert abs(p[5] - ref["log_prior"]) <= 1e-12 * max(1.0, abs(ref["log_prior"]))


def test_batched_thetas_equal_single_calls_bitwise(D):
    wl = W.config0()
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model)
    rng = np.random.default_rng(0)
    thetas = wl.theta[None] + 0.1 * rng.standard_normal((3, wl.dim_theta))
    fb, pb, _ = ws.fobj(thetas)
    singles = [ws.fobj(th)[0].item() for th in thetas]
    assert fb.cpu().tolist() == singles
    f2, _, _ = ws.fobj(thetas)
    assert f2.cpu().tolist() == fb.cpu().tolist()   # deterministic


def test_non_spd_theta_gives_minus_inf(D):
    """A theta whose Q_c is not positive definite cannot come from the
    parametrisation; force one through a huge negative log-precision that
    underflows the diagonal, and check f = -inf with a pivot report."""
    wl = W.config0()
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model)
    th = wl.theta.copy()
    th[0] = 400.0   # kappa^4 overflows to inf -> not a valid matrix
    f, parts, info = ws.fobj(th)
    torch.cuda.synchronize()
    assert f.item() == -math.inf


@pytest.mark.parametrize("sd", [0.3, 2.5])
def test_theta_prior_sd_and_mean(D, sd):
    """A prior on theta with sd != 1 and a mean away from the evaluation
    point: log p(theta) (the Gaussian density, constant included) and f_obj
    against the oracle, univariate and trivariate."""
    for wl in (W.config0(), W.scaled("tri_sd", 5, 4, 3, 2, 40, seed=4)):
        wl.theta_prior_sd = sd
        wl.theta_prior_mean = wl.theta + 0.2 * np.cos(np.arange(wl.dim_theta))
        ref = OF.fobj_parts(wl, wl.theta)
        model = D.Model.from_workload(wl)
        ws = D.Workspace(model)
        f, parts, info = ws.fobj(wl.theta)
        torch.cuda.synchronize()
        p = parts.cpu().numpy()[0]
        assert info.cpu().tolist() == [[0, 0]]
        assert abs(p[5] - ref["log_prior"]) <= 1e-12 * max(1.0, abs(ref["log_prior"]))
        scale = abs(ref["logdet_p"]) + abs(ref["logdet_c"])
        assert abs(f.item() - ref["f"]) <= 1e-10 * scale
