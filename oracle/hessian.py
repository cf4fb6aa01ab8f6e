"""CPU oracle -- the Hessian of f at the mode and the Gaussian approximation
of the hyperparameter marginals (Sec. II-C, marginal posteriors of the
hyperparameters).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in
``oracle/``.

The paper takes the negative Hessian of f at theta* by a second-order finite
difference scheme like the gradient's (Eq. 10) and uses it for a Gaussian
approximation of the marginals.  Read here as the standard central second
differences with one step h on the internal theta:
    H_ii = (f(x + h e_i) - 2 f(x) + f(x - h e_i)) / h^2,
    H_ij = (f(x + h e_i + h e_j) - f(x + h e_i - h e_j)
            - f(x - h e_i + h e_j) + f(x - h e_i - h e_j)) / (4 h^2),
2 d^2 + 1 independent evaluations; the Gaussian approximation has
covariance (-H)^{-1}, its marginal standard deviations the square roots of
the diagonal.
"""
from __future__ import annotations

import numpy as np


def hessian_stencil(theta, h: float = 1e-3) -> np.ndarray:
    """Rows: theta; theta + h e_i, theta - h e_i (i = 0..d-1); then for each
    pair i < j the four corners (+,+), (+,-), (-,+), (-,-)."""
    x = np.asarray(theta, np.float64)
    d = x.shape[0]
    E = np.eye(d) * h
    pts = [x.copy()]
    for i in range(d):
        pts.append(x + E[i])
        pts.append(x - E[i])
    for i in range(d):
        for j in range(i + 1, d):
            pts.append(x + E[i] + E[j])
            pts.append(x + E[i] - E[j])
            pts.append(x - E[i] + E[j])
            pts.append(x - E[i] - E[j])
    return np.stack(pts)


def hessian_from_values(values, d: int, h: float = 1e-3) -> np.ndarray:
    """The second differences above from the values at hessian_stencil."""
    v = np.asarray(values, np.float64)
    H = np.empty((d, d))
    f0 = v[0]
    for i in range(d):
        H[i, i] = (v[1 + 2 * i] - 2.0 * f0 + v[2 + 2 * i]) / (h * h)
    k = 1 + 2 * d
    for i in range(d):
        for j in range(i + 1, d):
            pp, pm, mp, mm = v[k:k + 4]
            H[i, j] = H[j, i] = (pp - pm - mp + mm) / (4.0 * h * h)
            k += 4
    return H


def hessian(f, theta, h: float = 1e-3) -> np.ndarray:
    pts = hessian_stencil(theta, h)
    return hessian_from_values([f(p) for p in pts], len(theta), h)


def gaussian_marginal_sd(H) -> np.ndarray:
    """Marginal standard deviations of the Gaussian with covariance (-H)^{-1}
    (H: Hessian of a log density at its mode, negative definite)."""
    C = np.linalg.inv(-np.asarray(H, np.float64))
    return np.sqrt(np.diag(C))
