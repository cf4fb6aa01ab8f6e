"""The largest block the library accepts: one response on a 100 x 100 mesh
(b = 10000, padded to 10048; the assembly builds a column of a diagonal and
a sub-diagonal block in LDS, 2 * 10048 + 64 doubles <= 160 KiB).

Without observations Q_c = Q_p = tau_u (T (x) Q_s) (+ the fixed effects'
prior), whose log-determinant and marginal variances have closed forms at
any size (Q_s: 2-D DCT spectrum (kappa^2 + l_i + l_j)^2 of the Neumann
grid Laplacian; T: unit-variance AR1, log|T| = -(nt-1) log(1 - rho^2),
diag(T^-1) = 1), so every one of the N variances is checked, and
f = log p(theta).  With observations the two elimination orders must agree
to rounding.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import model as OM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NX = 100


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_06938_amd import dalia
    dalia.lib()
    return dalia


def _dct_eigs(nx):
    return 2.0 - 2.0 * np.cos(np.pi * np.arange(nx) / nx)


def _qs_closed(nx, kappa):
    """log|Q_s| and diag(Q_s^-1) (node s = iy nx + ix) from the DCT."""
    lam = _dct_eigs(nx)
    ev = (kappa ** 2 + lam[:, None] + lam[None, :]) ** 2
    i = np.arange(nx)[:, None]
    k = np.arange(nx)[None, :]
    V = np.cos(np.pi * k * (i + 0.5) / nx) * math.sqrt(2.0 / nx)
    V[:, 0] = 1.0 / math.sqrt(nx)
    V2 = V * V
    diag = np.einsum("xk,yl,kl->yx", V2, V2, 1.0 / ev).ravel()
    return float(np.sum(np.log(ev))), diag


@pytest.mark.parametrize("two_sided", [False, True])
def test_largest_block_without_observations_matches_closed_forms(D, two_sided):
    wl = W.scaled("max_noobs", NX, 4, 1, 2, 0, seed=1)
    th = wl.theta + np.array([0.1, -0.2, 0.3, 0.0])
    p = OM.theta_to_params(th, 1)
    kappa, rho, tau_u = p["kappa"][0], p["rho"][0], p["tau_u"]
    ns, nt, a = wl.ns, wl.nt, wl.a
    ld_qs, dq = _qs_closed(NX, kappa)
    logdet = (ns * nt * math.log(tau_u) - ns * (nt - 1) * math.log(1.0 - rho * rho)
              + nt * ld_qs + a * math.log(wl.prior_fixed))
    var = np.concatenate([np.tile(dq / tau_u, nt), np.full(a, 1.0 / wl.prior_fixed)])
    model = D.Model.from_workload(wl)
    assert model.b == 10000 and model.bp == 10048
    ws = D.Workspace(model, selinv=True, two_sided=two_sided, fold_inverse=two_sided)
    f, parts, info = ws.fobj(th)
    mu = ws.mean()
    v = ws.selinv()
    torch.cuda.synchronize()
    pr = parts.cpu().numpy()[0]
    print(f"N={wl.N} logdet {pr[1]:.10f} closed {logdet:.10f}", flush=True)
    assert info.cpu().tolist() == [[0, 0]]
    assert abs(pr[1] - logdet) <= 1e-10 * abs(logdet)
    assert abs(pr[2] - logdet) <= 1e-10 * abs(logdet)
    assert not np.any(mu.cpu().numpy())
    np.testing.assert_allclose(v.cpu().numpy(), var, rtol=1e-9)
    lp = OM.log_prior_theta(th, wl.theta_prior_mean, wl.theta_prior_sd)
    assert abs(f.item() - lp) <= 1e-9 * abs(logdet)
    del ws


def test_largest_block_with_observations_orders_agree(D):
    wl = W.scaled("max_obs", NX, 4, 1, 2, 40_000, seed=2)
    model = D.Model.from_workload(wl)
    out = []
    for kw in ({}, {"two_sided": True, "fold_inverse": True}):
        ws = D.Workspace(model, selinv=True, **kw)
        f, parts, info = ws.fobj(wl.theta)
        v = ws.selinv()
        torch.cuda.synchronize()
        assert info.cpu().tolist() == [[0, 0]]
        out.append((f.item(), parts.cpu().numpy()[0], v.cpu().numpy()))
        del ws
    (f0, p0, v0), (f1, p1, v1) = out
    assert np.isfinite(f0) and abs(f1 - f0) <= 1e-11 * (abs(p0[1]) + abs(p0[2]))
    assert abs(p1[2] - p0[2]) <= 1e-12 * abs(p0[2])
    np.testing.assert_allclose(v1, v0, rtol=1e-10)
    assert np.all(v0 > 0) and p0[7] <= 1e-12
