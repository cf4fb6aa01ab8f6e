"""CPU oracle -- the Hessian of f at the mode and the Gaussian approximation
of the hyperparameter marginals (Sec. III, marginal posteriors of the
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

The paper's more accurate alternative reparametrises theta by the
eigenvectors of the Hessian to allow skewed marginals, citing Martins et
al. (2013), and gives no formula.  Read as that reference's split-normal
correction: with -H = V diag(lambda) V^T and A = V diag(lambda)^{-1/2},
theta(z) = theta* + A z makes the Gaussian approximation standard in z;
along each axis k, f is evaluated at z = +delta e_k and -delta e_k (2 d
evaluations), and the scale on each side is the one that a Gaussian with
that drop of f would have,
    sigma_k^{+-} = delta / sqrt(2 (f(theta*) - f(theta(+-delta e_k)))),
which is 1 on both sides when f is quadratic.  The asymmetric standard
deviations of theta_j combine the axes linearly: its upper side takes, on
every axis k, the side of z_k that raises theta_j (the sign of A_jk),
    s_j^+ = sqrt(sum_k A_jk^2 (sigma_k^{sign A_jk})^2),
and s_j^- the opposite sides; for a quadratic f both equal the Gaussian
marginal standard deviation.
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


def eigen_axes(H):
    """A = V diag(lambda)^{-1/2} for -H = V diag(lambda) V^T (eigenvalues in
    ascending order, each eigenvector's sign fixed so that its entry of
    largest magnitude is positive)."""
    lam, V = np.linalg.eigh(-np.asarray(H, np.float64))
    if lam.min() <= 0.0:
        raise ValueError("the Hessian is not negative definite")
    for k in range(V.shape[1]):
        if V[np.argmax(np.abs(V[:, k])), k] < 0:
            V[:, k] = -V[:, k]
    return V / np.sqrt(lam)[None, :]


def skew_points(theta_star, A, delta: float = 1.0) -> np.ndarray:
    """Rows: theta* + delta A e_k, theta* - delta A e_k for k = 0..d-1."""
    x = np.asarray(theta_star, np.float64)
    rows = []
    for k in range(A.shape[1]):
        rows.append(x + delta * A[:, k])
        rows.append(x - delta * A[:, k])
    return np.stack(rows)


def skew_scales(f_star: float, values, delta: float = 1.0):
    """(sigma^+, sigma^-) per axis from f at skew_points (same order)."""
    v = np.asarray(values, np.float64)
    drop_p = f_star - v[0::2]
    drop_m = f_star - v[1::2]
    if np.any(drop_p <= 0.0) or np.any(drop_m <= 0.0):
        raise ValueError("f does not drop along every axis: theta* is not a mode")
    return delta / np.sqrt(2.0 * drop_p), delta / np.sqrt(2.0 * drop_m)


def asymmetric_sd(A, sig_plus, sig_minus):
    """(s^+, s^-) of every theta_j from the axis scales."""
    A = np.asarray(A, np.float64)
    up = np.where(A >= 0.0, sig_plus[None, :], sig_minus[None, :])
    dn = np.where(A >= 0.0, sig_minus[None, :], sig_plus[None, :])
    return (np.sqrt(np.sum(A * A * up * up, axis=1)),
            np.sqrt(np.sum(A * A * dn * dn, axis=1)))
