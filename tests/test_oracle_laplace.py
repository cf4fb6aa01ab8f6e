"""Pins of the oracle's f_obj for a non-Gaussian (Poisson) likelihood: the
Laplace approximation at the inner mode (Eq. 3, 4, 8).

* The Gaussian likelihood through the same Newton/Laplace routine must give
  the Gaussian oracle's f_obj and mean (which are pinned on their own):
  this checks every term of the formula (both half log-determinants, the
  prior quadratic form, the likelihood) and the Newton update.
* The Laplace value against the log marginal likelihood by quadrature on
  tiny problems (one and two latent variables, large counts, where the
  Laplace error is O(1 / count)).
* The inner mode is a stationary point of log l - 1/2 x^T Q_p x (brute-force
  central differences).
* The Poisson log-likelihood against its closed forms at y = 0, 1, 3.
* The theta layout without the noise precision.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import fobj as OF
from oracle import laplace as OL
from oracle import model as OM


def test_poisson_loglik_closed_forms():
    eta = np.array([-0.5, 0.3, 1.2])
    assert OL.Poisson([0, 0, 0]).loglik(eta) == pytest.approx(-np.exp(eta).sum(), rel=1e-14)
    assert OL.Poisson([1, 1, 1]).loglik(eta) == pytest.approx(
        (eta - np.exp(eta)).sum(), rel=1e-14)
    assert OL.Poisson([3.0]).loglik(np.array([0.7])) == pytest.approx(
        3 * 0.7 - math.exp(0.7) - math.log(6.0), rel=1e-14)


@pytest.mark.parametrize("make", [W.config0,
                                  lambda: W.scaled("tri", 5, 4, 3, 2, 40, seed=4),
                                  lambda: W.scaled("d", 6, 5, 1, 2, 80, seed=5,
                                                   model="diffusion")])
def test_gaussian_special_case_reproduces_gaussian_fobj(make):
    wl = make()
    theta = wl.theta + 0.05 * np.sin(np.arange(wl.dim_theta) + 1.0)
    ref = OF.fobj_parts(wl, theta)
    Qp = OM.prior_precision(wl, theta)
    A = OM.design_matrix(wl)
    lik = OL.Gaussian(OM.observations(wl), OM.noise_precision(wl, theta))
    got = OL.laplace_parts(Qp, A, lik, ref["log_prior"], wl.nv * wl.nr)
    assert got["converged"] and got["newton_steps"] == 2   # exact mean, then a null step
    assert got["halvings"] == [0, 0]
    assert got["f"] == pytest.approx(ref["f"], rel=1e-11, abs=1e-9)
    np.testing.assert_allclose(got["mu"], ref["mu"], rtol=1e-9, atol=1e-11)
    assert got["logdet_c"] == pytest.approx(ref["logdet_c"], rel=1e-12)


def _log_marginal_by_quadrature(Qp, A, y, half_width=9.0, n=1601):
    """log of the integral of prod Poisson(y | exp(A x)) N(x | 0, Qp^-1) over
    x (one or two dimensions), by a Riemann sum on a grid around the
    posterior mode that reaches half_width posterior standard deviations."""
    Qp = np.asarray(Qp, np.float64)
    d = Qp.shape[0]
    lik = OL.Poisson(y)
    x, _, ok, _ = OL.inner_mode(sp.csr_matrix(Qp), sp.csr_matrix(A), lik)
    assert ok
    Qc = Qp + A.T @ np.diag(np.exp(A @ x)) @ A
    sd = np.sqrt(np.diag(np.linalg.inv(Qc)))
    axes = [np.linspace(x[i] - half_width * sd[i], x[i] + half_width * sd[i], n)
            for i in range(d)]
    grids = np.meshgrid(*axes, indexing="ij")
    pts = np.stack([g.ravel() for g in grids], axis=1)
    eta = pts @ A.T
    ll = (eta * y[None, :] - np.exp(eta)).sum(axis=1) - sum(math.lgamma(v + 1) for v in y)
    sign, logdet = np.linalg.slogdet(Qp)
    lprior = (-0.5 * d * math.log(2 * math.pi) + 0.5 * logdet
              - 0.5 * np.einsum("ki,ij,kj->k", pts, Qp, pts))
    v = ll + lprior
    vmax = v.max()
    cell = np.prod([ax[1] - ax[0] for ax in axes])
    return vmax + math.log(np.exp(v - vmax).sum() * cell)


def test_laplace_against_quadrature_one_latent():
    rng = np.random.default_rng(0)
    m = 20
    A = np.ones((m, 1))
    y = rng.poisson(math.exp(2.0), size=m).astype(np.float64)
    Qp = np.array([[2.0]])
    exact = _log_marginal_by_quadrature(Qp, A, y, n=20001)
    lap = OL.laplace_parts(sp.csr_matrix(Qp), sp.csr_matrix(A), OL.Poisson(y), 0.0)
    err = lap["f"] - exact
    print("one latent: laplace", lap["f"], "quadrature", exact, "error", err)
    assert abs(err) < 5e-3          # O(1 / sum y), sum y ~ 150
    # fewer counts: a larger Laplace error, of the expected size
    y2 = rng.poisson(1.0, size=4).astype(np.float64)
    A2 = np.ones((4, 1))
    err2 = (OL.laplace_parts(sp.csr_matrix(Qp), sp.csr_matrix(A2), OL.Poisson(y2), 0.0)["f"]
            - _log_marginal_by_quadrature(Qp, A2, y2, n=20001))
    assert abs(err) < abs(err2) < 0.2


def test_laplace_against_quadrature_two_latent():
    rng = np.random.default_rng(1)
    rows = np.array([[1.0, 0.0], [0.0, 1.0], [0.5, 0.5], [0.8, -0.3]])
    A = np.repeat(rows, 10, axis=0)
    x_true = np.array([2.2, 1.6])
    y = rng.poisson(np.exp(A @ x_true)).astype(np.float64)
    Qp = np.array([[2.0, -0.8], [-0.8, 1.5]])
    exact = _log_marginal_by_quadrature(Qp, A, y, n=801)
    lap = OL.laplace_parts(sp.csr_matrix(Qp), sp.csr_matrix(A), OL.Poisson(y), 0.0)
    err = lap["f"] - exact
    print("two latent: laplace", lap["f"], "quadrature", exact, "error", err)
    assert abs(err) < 5e-3
    # the same with A's columns swapped is a different problem: a transposed
    # or permuted design would not pass
    lap_swapped = OL.laplace_parts(sp.csr_matrix(Qp), sp.csr_matrix(A[:, ::-1].copy()),
                                   OL.Poisson(y), 0.0)
    assert abs(lap_swapped["f"] - exact) > 0.1


@pytest.mark.parametrize("nv", [1, 3])
def test_inner_mode_is_stationary(nv):
    wl = W.scaled("st", 4, 3, nv, 2, 60, seed=7, likelihood="poisson")
    Qp = OM.prior_precision(wl, wl.theta)
    A = OM.design_matrix(wl)
    lik = OL.likelihood_of(wl, wl.theta)
    x, steps, ok, halv = OL.inner_mode(Qp, A, lik, wl.nv * wl.nr)
    assert ok
    h = 1e-5
    grad = np.empty_like(x)
    for i in range(x.shape[0]):
        e = np.zeros_like(x)
        e[i] = h
        grad[i] = (OL.inner_objective(Qp, A, lik, x + e)
                   - OL.inner_objective(Qp, A, lik, x - e)) / (2 * h)
    scale = np.abs(A.T @ lik.y).max()
    print("steps", steps, "halvings", halv, "max |grad|", np.abs(grad).max(), "scale", scale)
    assert np.abs(grad).max() <= 1e-6 * scale
    # the closed-form gradient vanishes there too
    g = A.T @ lik.grad(A @ x) - Qp @ x
    assert np.abs(g).max() <= 1e-9 * scale
    # and x* is a maximum: moving along any coordinate lowers the objective
    h0 = OL.inner_objective(Qp, A, lik, x)
    for i in range(0, x.shape[0], 7):
        e = np.zeros_like(x)
        e[i] = 1e-3
        assert OL.inner_objective(Qp, A, lik, x + e) < h0


def test_damping_is_needed_and_every_step_ascends():
    """A full Newton step from x = 0 overshoots on this trivariate count
    workload; the damped iteration halves it and still converges quickly."""
    wl = W.scaled("p", 8, 5, 3, 2, 200, seed=3, likelihood="poisson")
    parts = OF.fobj_parts(wl, wl.theta)
    assert parts["converged"] and parts["halvings"][0] >= 1
    assert parts["newton_steps"] <= 12
    Qp = OM.prior_precision(wl, wl.theta)
    A = OM.design_matrix(wl)
    lik = OL.likelihood_of(wl, wl.theta)
    x0 = np.zeros(Qp.shape[0])
    Dv = lik.neg_hess(A @ x0)
    Qc = (Qp + A.T @ (A.multiply(Dv[:, None]))).tocsr()
    from oracle.linalg import factor
    x_full = factor(Qc, 6).solve(A.T @ (lik.grad(A @ x0) + Dv * (A @ x0)))
    assert OL.inner_objective(Qp, A, lik, x_full) < OL.inner_objective(Qp, A, lik, x0)


def test_poisson_theta_layout():
    assert OM.theta_dim(1, "poisson") == 3 and OM.theta_dim(3, "poisson") == 12
    wl = W.scaled("p", 5, 4, 3, 2, 40, seed=2, likelihood="poisson")
    assert wl.dim_theta == 12 and wl.theta.shape == (12,)
    g = W.scaled("g", 5, 4, 3, 2, 40, seed=2)
    # the prior does not involve the noise precisions: dropping them from a
    # Gaussian theta gives the Poisson workload's Q_p for the same values
    np.testing.assert_array_equal(
        OM.prior_precision(wl, g.theta[:12]).toarray(),
        OM.prior_precision(g, g.theta).toarray())
    assert OM.theta_to_params(wl.theta, 3, likelihood="poisson")["tau_y"] is None
    with pytest.raises(ValueError):
        OM.noise_precision(wl, wl.theta)
    with pytest.raises(ValueError):
        OM.theta_to_params(wl.theta, 3, likelihood="binomial")
    y = OM.observations(wl)
    assert np.all(y >= 0) and np.all(y == np.round(y))
