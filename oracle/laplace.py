"""CPU FP64 oracle -- f_obj(theta) for a non-Gaussian likelihood (Section
II-A, conditional Gaussian distribution, Eq. 3, 4 and 8).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in
``oracle/``.

For a likelihood that is not Gaussian, p_G is the Gaussian built from a
second-order expansion of the log-likelihood, D is the negative Hessian of
the log-likelihood at x (Eq. 4), and p_G is only an approximation, so its
mean has to be found by an inner search.  The paper sketches this and fixes
no algorithm; read here as the standard Laplace approximation:

* the mode x* of h(x) = log l(y | A x) - 1/2 x^T Q_p x (log p(x | theta)
  up to a constant) by damped Newton from x = 0: with eta = A x,
  g = d log l / d eta and D = -d^2 log l / d eta^2 (diagonal, one entry per
  observation),
      Q_c(x) = Q_p + A^T D A,     x_N = Q_c(x)^{-1} A^T (g + D eta),
  the step x + alpha (x_N - x) with the first alpha in 1, 1/2, 1/4, ...
  (at most 30 halvings) for which h does not fall, up to rounding:
  h(new) >= h(x) - 1e-12 (1 + |h(x)|).  A full Newton step from x = 0
  overshoots badly for counts (the exponential turns a too-large eta into
  enormous weights and Newton then walks back about one unit per step);
  since h is concave the halving keeps every step an ascent.  Stop after a
  full step (alpha = 1) with max |x_N - x| <= tol (1 + max |x_N|),
  tol = 1e-9; at most 40 steps (not converged, or no acceptable alpha:
  f = -inf);
* f_obj of Eq. 8 at x = x*, with p_G the Gaussian of mean x* and precision
  Q_c(x*) (assembled and factored again at x*):
      f = log p(theta) + log l(y | x*) + 1/2 log|Q_p| - 1/2 x*^T Q_p x*
          - 1/2 log|Q_c(x*)|,
  the (2 pi)^{-N/2} of Eq. 1 and Eq. 3 cancelling as in the Gaussian case.

Poisson counts with the log link: log l = sum_i y_i eta_i - exp(eta_i)
- log(y_i!), g = y - exp(eta), D = diag(exp(eta)).

For a Gaussian likelihood the same routine takes one Newton step to the
exact mean (D = tau, g + D eta = tau y) and reproduces ``fobj.fobj_parts``.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import gammaln

from . import model as M
from .linalg import factor, NotSPD

NEWTON_TOL = 1e-9
NEWTON_MAX = 40
NEWTON_HALVINGS = 30
ASCENT_SLACK = 1e-12


class Poisson:
    """Counts y with log link."""

    def __init__(self, y):
        self.y = np.asarray(y, np.float64)

    def loglik(self, eta) -> float:
        return float(np.sum(self.y * eta - np.exp(eta) - gammaln(self.y + 1.0)))

    def grad(self, eta):
        return self.y - np.exp(eta)

    def neg_hess(self, eta):
        return np.exp(eta)


class Gaussian:
    """y_i ~ N(eta_i, 1/tau_i) (Eq. 2), the special case that has no
    approximation in it."""

    def __init__(self, y, tau):
        self.y = np.asarray(y, np.float64)
        self.tau = np.asarray(tau, np.float64) * np.ones_like(self.y)

    def loglik(self, eta) -> float:
        r = self.y - eta
        return float(np.sum(0.5 * np.log(self.tau) - 0.5 * math.log(2 * math.pi)
                            - 0.5 * self.tau * r * r))

    def grad(self, eta):
        return self.tau * (self.y - eta)

    def neg_hess(self, eta):
        return self.tau.copy()


def inner_objective(Qp, A, lik, x) -> float:
    """h(x) = log l(y | A x) - 1/2 x^T Q_p x."""
    return lik.loglik(A @ x) - 0.5 * float(x @ (Qp @ x))


def inner_mode(Qp, A, lik, a: int = 0, method: str = "auto",
               tol: float = NEWTON_TOL, max_iter: int = NEWTON_MAX):
    """Damped Newton for the mode of h from x = 0.  Returns (x, steps,
    converged, halvings per step)."""
    x = np.zeros(Qp.shape[0])
    hx = inner_objective(Qp, A, lik, x)
    halvings = []
    for k in range(1, max_iter + 1):
        eta = A @ x
        Dv = lik.neg_hess(eta)
        Qc = (Qp + A.T @ (A.multiply(Dv[:, None]))).tocsr()
        x_N = factor(Qc, a, method).solve(A.T @ (lik.grad(eta) + Dv * eta))
        alpha, nh = 1.0, 0
        while True:
            x_t = x + alpha * (x_N - x)
            h_t = inner_objective(Qp, A, lik, x_t)
            if np.isfinite(h_t) and h_t >= hx - ASCENT_SLACK * (1.0 + abs(hx)):
                break
            if nh == NEWTON_HALVINGS:
                return x, k, False, halvings
            alpha *= 0.5
            nh += 1
        halvings.append(nh)
        step = float(np.max(np.abs(x_N - x)))
        x, hx = x_t, h_t
        if nh == 0 and step <= tol * (1.0 + float(np.max(np.abs(x_N)))):
            return x, k, True, halvings
    return x, max_iter, False, halvings


def laplace_parts(Qp, A, lik, log_prior: float, a: int = 0, method: str = "auto",
                  tol: float = NEWTON_TOL, max_iter: int = NEWTON_MAX) -> dict:
    """The parts of f_obj at the inner mode for given Q_p, A and likelihood."""
    N = Qp.shape[0]
    out = dict(N=N, m=A.shape[0])
    try:
        Fp = factor(Qp, a, method)
        x, steps, ok, halvings = inner_mode(Qp, A, lik, a, method, tol, max_iter)
        eta = A @ x
        Dv = lik.neg_hess(eta)
        Qc = (Qp + A.T @ (A.multiply(Dv[:, None]))).tocsr()
        Fc = factor(Qc, a, method)
    except NotSPD:
        out.update(f=-math.inf, spd=False)
        return out
    logdet_p = Fp.logdet()
    logdet_c = Fc.logdet()
    quad_p = float(x @ (Qp @ x))
    log_lik = lik.loglik(eta)
    f = log_prior + log_lik + 0.5 * logdet_p - 0.5 * quad_p - 0.5 * logdet_c
    if not ok or not np.isfinite(f):
        f = -math.inf
    out.update(f=f, spd=True, converged=ok, newton_steps=steps, halvings=halvings,
               logdet_p=logdet_p, logdet_c=logdet_c, quad_p=quad_p,
               log_lik=log_lik, log_prior=log_prior, mu=x, D=Dv, Qp=Qp, Qc=Qc, Fp=Fp, Fc=Fc,
               r=A.T @ (lik.grad(eta) + Dv * eta))
    return out


def likelihood_of(wl, theta):
    y = M.observations(wl)
    if M.likelihood_family(wl) == "poisson":
        return Poisson(y)
    return Gaussian(y, M.noise_precision(wl, theta))


def fobj_parts_laplace(wl, theta, method: str = "auto") -> dict:
    """f_obj(theta) and its parts for a workload of any likelihood."""
    theta = np.asarray(theta, np.float64)
    Qp = M.prior_precision(wl, theta)
    A = M.design_matrix(wl)
    lp = M.log_prior_theta(theta, wl.theta_prior_mean, wl.theta_prior_sd)
    out = laplace_parts(Qp, A, likelihood_of(wl, theta), lp, wl.nv * wl.nr, method)
    if out["spd"]:
        out["quad_obs"] = -2.0 * out["log_lik"]
    return out
