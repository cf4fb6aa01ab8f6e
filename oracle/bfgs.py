"""CPU oracle -- mode search over theta (Eq. 9) with the central-difference
gradient of Eq. 10.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in
``oracle/``.

The paper minimises -f_obj with BFGS (Nocedal & Wright) and approximates
each partial derivative by a central difference with step h; the
2*dim(theta)+1 evaluations of one gradient are independent.  The paper does
not fix the line search, the initial inverse Hessian or the stopping rule;
read here as: the search direction is capped at length max_step (theta holds
log-scale parameters, so a unit step already changes a scale by e), the
initial inverse Hessian is the identity rescaled by y^T s / y^T y before the
first update (Nocedal & Wright, Sec. 6.1), Armijo backtracking (c1 = 1e-4,
halving), one restart along the steepest-descent direction when the line
search fails, and stop when the relative change of f is at most ftol or the
largest gradient component is at most gtol.
"""
from __future__ import annotations

import numpy as np


def fd_stencil(theta, h: float = 1e-3) -> np.ndarray:
    """theta, theta + h e_1, theta - h e_1, theta + h e_2, ... (rows)."""
    theta = np.asarray(theta, np.float64)
    d = theta.shape[0]
    pts = [theta.copy()]
    for i in range(d):
        e = np.zeros(d)
        e[i] = h
        pts.append(theta + e)
        pts.append(theta - e)
    return np.stack(pts)


def central_gradient_from_values(values, h: float = 1e-3) -> np.ndarray:
    """Eq. 10 from the values at fd_stencil points: (f(+h e_i) - f(-h e_i))/2h."""
    v = np.asarray(values, np.float64)
    return (v[1::2] - v[2::2]) / (2.0 * h)


def central_gradient(f, theta, h: float = 1e-3) -> np.ndarray:
    pts = fd_stencil(theta, h)
    return central_gradient_from_values([f(p) for p in pts], h)


def _capped(p, max_step):
    nrm = float(np.linalg.norm(p))
    return p * (max_step / nrm) if nrm > max_step else p


def bfgs_minimize(fun_and_grad, x0, max_iter: int = 100, ftol: float = 1e-6,
                  gtol: float = 1e-4, c1: float = 1e-4, max_halvings: int = 30,
                  max_step: float = 1.0):
    """Minimise a smooth function given f and its gradient at a point.

    fun_and_grad(x) -> (f, g).  Inverse-Hessian BFGS update
    H <- (I - r s y^T) H (I - r y s^T) + r s s^T, r = 1/(y^T s), skipped when
    y^T s <= 0.  Returns (x, f, history) with history a list of dicts."""
    x = np.asarray(x0, np.float64).copy()
    f, g = fun_and_grad(x)
    n = x.shape[0]
    H = np.eye(n)
    first = True
    hist = [dict(x=x.copy(), f=f, gnorm=float(np.max(np.abs(g))), evals=1)]
    for it in range(max_iter):
        if np.max(np.abs(g)) <= gtol:
            break
        p = -H @ g
        if g @ p >= 0:          # not a descent direction: restart
            H = np.eye(n)
            p = -g
        accepted = False
        for attempt in range(2):
            p = _capped(p, max_step)
            alpha = 1.0
            for _ in range(max_halvings):
                xn = x + alpha * p
                fn, gn = fun_and_grad(xn)
                if np.isfinite(fn) and fn <= f + c1 * alpha * (g @ p):
                    accepted = True
                    break
                alpha *= 0.5
            if accepted or attempt == 1:
                break
            H = np.eye(n)        # one restart along steepest descent
            p = -g
        if not accepted:
            break
        s = xn - x
        y = gn - g
        ys = y @ s
        if ys > 1e-12:
            if first:
                H = (ys / (y @ y)) * np.eye(n)
                first = False
            r = 1.0 / ys
            I = np.eye(n)
            H = (I - r * np.outer(s, y)) @ H @ (I - r * np.outer(y, s)) + r * np.outer(s, s)
        rel = abs(fn - f) / max(1.0, abs(f))
        x, f, g = xn, fn, gn
        hist.append(dict(x=x.copy(), f=f, gnorm=float(np.max(np.abs(g)))))
        if rel <= ftol:
            break
    return x, f, hist
