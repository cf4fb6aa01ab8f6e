"""CPU FP64 oracle -- the objective f_obj(theta) of Eq. 8.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in
``oracle/``.

For a Gaussian likelihood the Gaussian approximation p_G is exact (Eq. 3),
its precision is Q_c = Q_p + A^T D A (Eq. 4) and its mean solves
Q_c mu = A^T D y.  The four terms of Eq. 8 are evaluated at x = mu, each
written out from its density:

  log p(theta)              Gaussian prior on internal theta
  log l(y | theta, x)       sum_j [m_j/2 log tau_j - m_j/2 log 2pi
                                   - tau_j/2 |y_j - A_j x|^2]      (Eq. 2)
  log p(x | theta)          -N/2 log 2pi + 1/2 log|Q_p| - 1/2 x^T Q_p x (Eq. 1)
  log p_G(x | theta, y)     -N/2 log 2pi + 1/2 log|Q_c|
                            - 1/2 (x-mu)^T Q_c (x-mu)                  (Eq. 3)
"""
from __future__ import annotations

import math

import numpy as np

from . import model as M
from .linalg import factor, NotSPD


def fobj_parts(wl, theta, method: str = "auto", x=None,
               return_factors: bool = False) -> dict:
    """All parts of f_obj(theta) at x (default x = mu).  Returns -inf for f
    and ``spd=False`` when Q_p or Q_c is not positive definite.  Workloads of
    a non-Gaussian likelihood go to ``laplace.fobj_parts_laplace`` (x = the
    inner mode; a given x is not supported there)."""
    if M.likelihood_family(wl) != "gaussian":
        if x is not None:
            raise ValueError("x is the inner mode for a non-Gaussian likelihood")
        from .laplace import fobj_parts_laplace
        return fobj_parts_laplace(wl, theta, method)
    theta = np.asarray(theta, np.float64)
    Qp = M.prior_precision(wl, theta)
    A = M.design_matrix(wl)
    d = M.noise_precision(wl, theta)
    y = M.observations(wl)
    Qc = (Qp + A.T @ (A.multiply(d[:, None]))).tocsr()
    a = wl.nv * wl.nr
    N = Qp.shape[0]
    m = y.shape[0]
    out = dict(N=N, m=m)
    try:
        Fp = factor(Qp, a, method)
        Fc = factor(Qc, a, method)
    except NotSPD:
        out.update(f=-math.inf, spd=False)
        return out
    r = A.T @ (d * y)
    mu = Fc.solve(r)
    xx = mu if x is None else np.asarray(x, np.float64)

    logdet_p = Fp.logdet()
    logdet_c = Fc.logdet()
    quad_p = float(xx @ (Qp @ xx))
    resid = y - A @ xx
    quad_obs = float(np.sum(d * resid * resid))
    dm = xx - mu
    quad_c = float(dm @ (Qc @ dm))

    log_prior = M.log_prior_theta(theta, wl.theta_prior_mean,
                                  wl.theta_prior_sd)
    log_lik = float(0.5 * np.sum(np.log(d)) - 0.5 * m * math.log(2 * math.pi)
                    - 0.5 * quad_obs)
    log_px = -0.5 * N * math.log(2 * math.pi) + 0.5 * logdet_p - 0.5 * quad_p
    log_pg = -0.5 * N * math.log(2 * math.pi) + 0.5 * logdet_c - 0.5 * quad_c
    f = log_prior + log_lik + log_px - log_pg
    out.update(f=f, spd=True, logdet_p=logdet_p, logdet_c=logdet_c,
               quad_p=quad_p, quad_obs=quad_obs, log_prior=log_prior,
               log_lik=log_lik, log_px=log_px, log_pg=log_pg, mu=mu, r=r)
    if return_factors:
        out.update(Fp=Fp, Fc=Fc, Qp=Qp, Qc=Qc, A=A, d=d, y=y)
    return out


def fobj(wl, theta, method: str = "auto") -> float:
    return fobj_parts(wl, theta, method)["f"]


def marginal_variances(wl, theta, idx=None, method: str = "auto"):
    """diag(Q_c^{-1}) at model-order indices ``idx`` (all if None): the
    marginal variances of the latent field (Section III-A, selected
    inversion)."""
    Qp = M.prior_precision(wl, theta)
    Qc = M.conditional_precision(wl, theta, Qp=Qp)
    F = factor(Qc, wl.nv * wl.nr, method)
    if idx is None:
        if isinstance(F, type(None)):
            raise ValueError
        idx = np.arange(Qc.shape[0])
    return F.inv_diag(idx)
