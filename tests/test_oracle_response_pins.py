"""Pins of the oracle's multi-response observation operator and of its prior
on theta, against facts that do not come from the oracle.

With Lambda = I (every sigma_i = 1, every lambda_k = 0) the coregional prior
precision of Eq. 11 is block diagonal over the responses, the fixed effects
of each response have their own independent prior, and every observation row
touches only its own response's field and fixed effects (Eq. 2, 5).  The
joint model then separates into nv independent univariate models (unit
process scale): log-determinants, quadratic forms and f_obj - log p(theta)
are sums of the univariate values, and the conditional mean and marginal
variances are the univariate ones, response by response.  Each response gets
its own kappa, rho and tau_y, so a response <-> field swap, a misplaced
fixed-effect slot or a reordered tau_y changes at least one of them; the
planted-mistake tests below show that each of these slips fails.

The prior on theta (independent Gaussians on the internal parameters,
normalising constant included) is checked against scipy's normal density
with sd != 1, where an sd <-> sd^2 slip or a dropped constant shows.
"""
import math

import numpy as np
import pytest
import scipy.stats as st

import workloads as W
from oracle import fobj as F
from oracle import model as M

KAPPA = (0.5, 1.0, 2.0)
RHO = (0.6, 0.8, 0.9)
TAU_Y = (2.0, 4.0, 8.0)


def _phi(rho):
    return math.log((1 + rho) / (1 - rho))


def identity_lambda_case(nv=3, seed=7, nx=5, nt=4, nr=2, m_per=50):
    """A coregional workload and a theta with sigma = 1, lambda = 0 and
    distinct kappa_j, rho_j, tau_y_j."""
    wl = W.scaled("lambda_identity", nx, nt, nv, nr, m_per, seed=seed)
    theta = np.concatenate([np.log(KAPPA[:nv]), [_phi(r) for r in RHO[:nv]],
                            np.zeros(nv), np.zeros(nv * (nv - 1) // 2),
                            np.log(TAU_Y[:nv])])
    wl.theta_prior_mean = theta.copy()
    return wl, theta


def univariate_of(wl, j):
    """Response j of `wl` as a univariate workload (tau_u = 1) and its theta
    [log kappa_j, phi_j, log tau_u = 0, log tau_y_j]."""
    r = wl.responses[j]
    th = np.array([math.log(KAPPA[j]), _phi(RHO[j]), 0.0, math.log(TAU_Y[j])])
    u = W.Workload(name=f"resp{j}", nx=wl.nx, nt=wl.nt, nv=1, nr=wl.nr,
                   responses=[W.Response(r.t, r.nodes, r.w, r.X, r.y)],
                   theta=th, theta_prior_mean=th.copy(),
                   theta_prior_sd=wl.theta_prior_sd, prior_fixed=wl.prior_fixed)
    return u, th


def check_responses_separate(wl, theta):
    """Raise AssertionError unless the Lambda = I model equals its nv
    univariate parts (sums of scalars, concatenation of vectors)."""
    tri = F.fobj_parts(wl, theta)
    uni = [univariate_of(wl, j) for j in range(wl.nv)]
    parts = [F.fobj_parts(u, th) for u, th in uni]
    for key in ("logdet_p", "logdet_c", "quad_p", "quad_obs"):
        want = sum(p[key] for p in parts)
        assert abs(tri[key] - want) <= 1e-11 * max(1.0, abs(want)), (key, tri[key], want)
    want = sum(p["f"] - p["log_prior"] for p in parts)
    scale = abs(tri["logdet_p"]) + abs(tri["logdet_c"])
    assert abs((tri["f"] - tri["log_prior"]) - want) <= 1e-11 * scale, (tri["f"], want)
    # conditional mean and marginal variances, response by response
    nst, nr = wl.ns * wl.nt, wl.nr
    var_tri = F.marginal_variances(wl, theta)
    for j, (u, th) in enumerate(uni):
        idx = np.concatenate([j * nst + np.arange(nst),
                              wl.nv * nst + j * nr + np.arange(nr)])
        mu_j = parts[j]["mu"]
        np.testing.assert_allclose(tri["mu"][idx], mu_j, rtol=0,
                                   atol=1e-10 * np.abs(mu_j).max())
        np.testing.assert_allclose(var_tri[idx], F.marginal_variances(u, th),
                                   rtol=1e-10)


@pytest.mark.parametrize("nv", [2, 3])
def test_identity_lambda_separates_responses(nv):
    wl, theta = identity_lambda_case(nv)
    check_responses_separate(wl, theta)


def test_identity_lambda_separates_with_unequal_response_sizes():
    """Responses with different row counts (m_j differ), so that the
    likelihood constant and the row -> response map are exercised."""
    wl, theta = identity_lambda_case(3)
    for j, keep in enumerate((50, 31, 17)):
        r = wl.responses[j]
        wl.responses[j] = W.Response(r.t[:keep], r.nodes[:keep], r.w[:keep],
                                     r.X[:keep], r.y[:keep])
    check_responses_separate(wl, theta)


def test_identity_lambda_mixing_is_identity():
    """With sigma = 1 and lambda = 0, Eq. 5's Lambda is I, so the weight of
    Q^i in block (j, k) of Eq. 11 is 1 when i = j = k and 0 otherwise."""
    M3 = M.mixing_weights(np.ones(3), np.zeros(3))
    want = np.zeros((3, 3, 3))
    for i in range(3):
        want[i, i, i] = 1.0
    assert np.array_equal(M3, want)


# ---- planted mistakes: each must fail the separation check -------------------

def _swap_field_columns(A, wl, shift):
    """Move the field columns of response j to response (j + shift) mod nv."""
    nst, nv = wl.ns * wl.nt, wl.nv
    cols = np.arange(A.shape[1])
    new = cols.copy()
    for j in range(nv):
        jj = (j + shift) % nv
        new[j * nst:(j + 1) * nst] = jj * nst + np.arange(nst)
    return A[:, np.argsort(new)]


def _permute_fixed_columns(A, wl):
    """Fixed effect (j, r) stored at slot r*nv + j instead of j*nr + r."""
    nst, nv, nr = wl.ns * wl.nt, wl.nv, wl.nr
    new = np.arange(A.shape[1])
    for j in range(nv):
        for r in range(nr):
            new[nv * nst + j * nr + r] = nv * nst + r * nv + j
    return A[:, np.argsort(new)]


PLANTS = {
    "response_field_swap": lambda orig: (
        lambda wl: _swap_field_columns(orig(wl), wl, 1)),
    "fixed_effect_slots": lambda orig: (
        lambda wl: _permute_fixed_columns(orig(wl), wl)),
}


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_planted_design_matrix_mistake_fails(monkeypatch, plant):
    wl, theta = identity_lambda_case(3)
    check_responses_separate(wl, theta)  # the unplanted oracle passes
    monkeypatch.setattr(M, "design_matrix", PLANTS[plant](M.design_matrix))
    with pytest.raises(AssertionError):
        check_responses_separate(wl, theta)


def test_planted_tau_order_mistake_fails(monkeypatch):
    orig = M.noise_precision

    def reversed_tau(wl, theta):
        if wl.nv == 1:
            return orig(wl, theta)
        p = M.theta_to_params(theta, wl.nv, M.model_family(wl))
        tau = p["tau_y"][::-1]
        return np.concatenate([np.full(r.y.shape[0], tau[j])
                               for j, r in enumerate(wl.responses)])

    wl, theta = identity_lambda_case(3)
    monkeypatch.setattr(M, "noise_precision", reversed_tau)
    with pytest.raises(AssertionError):
        check_responses_separate(wl, theta)


# ---- the prior on theta ------------------------------------------------------

@pytest.mark.parametrize("sd", [0.3, 1.0, 2.5])
def test_log_prior_theta_is_gaussian_density(sd):
    rng = np.random.default_rng(11)
    for d in (4, 15):
        th = rng.standard_normal(d)
        mu = rng.standard_normal(d)
        want = float(np.sum(st.norm.logpdf(th, loc=mu, scale=sd)))
        got = M.log_prior_theta(th, mu, sd)
        assert abs(got - want) <= 1e-13 * max(1.0, abs(want)), (sd, d, got, want)


def test_fobj_uses_the_prior_sd():
    """Only log p(theta) depends on the prior's sd: f_obj(sd) - f_obj(1)
    is the difference of the two normal log densities."""
    wl = W.scaled("prior_sd", 5, 4, 3, 2, 40, seed=2)
    th = wl.theta + 0.2 * np.sin(np.arange(wl.dim_theta))
    f1 = F.fobj_parts(wl, th)["f"]
    wl.theta_prior_sd = 2.5
    f2 = F.fobj_parts(wl, th)["f"]
    dlp = float(np.sum(st.norm.logpdf(th, wl.theta_prior_mean, 2.5))
                - np.sum(st.norm.logpdf(th, wl.theta_prior_mean, 1.0)))
    assert abs((f2 - f1) - dlp) <= 1e-9 * max(1.0, abs(f1))


def test_planted_prior_variance_slip_fails(monkeypatch):
    """An sd used where sd^2 belongs (or the constant dropped) misses the
    normal density at sd != 1."""
    def slipped(theta, mean, sd):
        th = np.asarray(theta, np.float64)
        mu = np.asarray(mean, np.float64)
        return float(-0.5 * th.shape[0] * math.log(2 * math.pi * sd)
                     - 0.5 * np.sum((th - mu) ** 2) / sd)

    monkeypatch.setattr(M, "log_prior_theta", slipped)
    with pytest.raises(AssertionError):
        test_log_prior_theta_is_gaussian_density(2.5)
