"""Mode search over theta (Eq. 9) on top of the batched evaluator.

Two drivers minimise F(theta) = -f_obj(theta):

* ``fd_bfgs``: BFGS with the central-difference gradient of Eq. 10.  The
  2*dim+1 stencil points of one gradient are one batched evaluation pass;
  the line search evaluates a ladder of trial step lengths (1, 1/2, 1/4, ...)
  as one more pass and keeps the longest step with sufficient (Armijo)
  decrease.
* ``surrogate_bfgs``: the same, but between exact gradients a learned
  surrogate (the GPU MLP, trained online on every exact (theta, f) pair)
  supplies the gradient that sets the search direction and the secant
  update; every proposed point is still evaluated exactly, and the exact
  values alone decide acceptance.  When a surrogate step is rejected the
  driver falls back to an exact finite-difference step.

Host-side logic only (vectors of length dim theta); every f_obj value comes
from the library's kernels.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional

import numpy as np
import torch

from . import dalia as D


@dataclasses.dataclass
class Trace:
    theta: List[np.ndarray] = dataclasses.field(default_factory=list)
    f: List[float] = dataclasses.field(default_factory=list)        # F = -f_obj
    exact_evals: List[int] = dataclasses.field(default_factory=list)
    wall: List[float] = dataclasses.field(default_factory=list)
    kind: List[str] = dataclasses.field(default_factory=list)


class Evaluator:
    """Batched exact evaluation of F = -f_obj on one model (B instances)."""

    def __init__(self, model: "D.Model", batch: int, graph: bool = True):
        self.model = model
        self.B = batch
        self.ws = D.Workspace([model] * batch, graph=graph)
        self.dim = model.dim_theta
        self.count = 0
        self.archive_x: List[np.ndarray] = []
        self.archive_f: List[float] = []

    def __call__(self, thetas: np.ndarray) -> np.ndarray:
        thetas = np.atleast_2d(np.asarray(thetas, np.float64))
        f, _, _ = self.ws.fobj(thetas)
        vals = -f.cpu().numpy()
        self.count += thetas.shape[0]
        for t, v in zip(thetas, vals):
            if np.isfinite(v):
                self.archive_x.append(t.copy())
                self.archive_f.append(float(v))
        return vals


def fd_points(theta: np.ndarray, h: float) -> np.ndarray:
    d = theta.shape[0]
    E = np.eye(d) * h
    pts = np.empty((2 * d + 1, d))
    pts[0] = theta
    pts[1::2] = theta + E
    pts[2::2] = theta - E
    return pts


def fd_gradient(ev: Evaluator, theta: np.ndarray, h: float):
    v = ev(fd_points(theta, h))
    return v[0], (v[1::2] - v[2::2]) / (2.0 * h)


def _line_search(ev: Evaluator, theta, F0, g, p, c1=1e-4, ntrial=None):
    """Evaluate theta + alpha p for alpha = 1, 1/2, ... in one pass; return
    the longest step with F <= F0 + c1 alpha g.p, else (None, None, None)."""
    n = ntrial or ev.B
    alphas = 0.5 ** np.arange(n)
    vals = ev(theta[None, :] + alphas[:, None] * p[None, :])
    slope = float(g @ p)
    for a, v in zip(alphas, vals):
        if np.isfinite(v) and v <= F0 + c1 * a * slope:
            return a, theta + a * p, v
    return None, None, None


def _bfgs_update(H, s, y):
    ys = float(y @ s)
    if ys <= 1e-12:
        return H
    r = 1.0 / ys
    I = np.eye(H.shape[0])
    return (I - r * np.outer(s, y)) @ H @ (I - r * np.outer(y, s)) + r * np.outer(s, s)


def fd_bfgs(ev: Evaluator, theta0, h=1e-3, ftol=1e-6, gtol=1e-4, max_iter=100,
            f_target: Optional[float] = None, target_rtol: float = 1e-6) -> Trace:
    t0 = time.perf_counter()
    tr = Trace()
    x = np.asarray(theta0, np.float64).copy()
    F, g = fd_gradient(ev, x, h)
    H = np.eye(x.shape[0])

    def log(kind):
        tr.theta.append(x.copy()); tr.f.append(F); tr.exact_evals.append(ev.count)
        tr.wall.append(time.perf_counter() - t0); tr.kind.append(kind)

    log("start")
    for _ in range(max_iter):
        if f_target is not None and abs(F - f_target) <= target_rtol * abs(f_target):
            break
        if np.max(np.abs(g)) <= gtol:
            break
        p = -H @ g
        if g @ p >= 0:
            H = np.eye(x.shape[0])
            p = -g
        a, xn, Fn = _line_search(ev, x, F, g, p)
        if a is None:
            break
        Fn2, gn = fd_gradient(ev, xn, h)
        H = _bfgs_update(H, xn - x, gn - g)
        rel = abs(Fn2 - F) / max(1.0, abs(F))
        x, F, g = xn, Fn2, gn
        log("fd")
        if f_target is None and rel <= ftol:
            break
    return tr


class Surrogate:
    """Online MLP model of F over theta (inputs centred and scaled by the
    archive, output standardised), trained with the GPU kernels."""

    def __init__(self, dim: int, hidden=(256, 256, 256), max_batch=4096, seed=0):
        sizes = (dim, *hidden, 1)
        self.net = D.MLP(sizes, max_batch=max_batch)
        rng = np.random.default_rng(seed)
        flat = []
        for i, o in zip(sizes[:-1], sizes[1:]):
            flat.append(rng.standard_normal(o * i) / math.sqrt(i))
            flat.append(np.zeros(o))
        self.net.params.copy_(torch.from_numpy(np.concatenate(flat).astype(np.float32)))
        self.dim = dim
        self.mx = np.zeros(dim)
        self.sx = np.ones(dim)
        self.my = 0.0
        self.sy = 1.0

    def fit(self, X: np.ndarray, y: np.ndarray, steps=200, lr=2e-3):
        self.mx = X.mean(axis=0)
        self.sx = X.std(axis=0) + 1e-3
        self.my = float(y.mean())
        self.sy = float(y.std() + 1e-12)
        Xn = torch.from_numpy(((X - self.mx) / self.sx).astype(np.float32)).cuda()
        yn = torch.from_numpy(((y - self.my) / self.sy).astype(np.float32)).cuda()
        for _ in range(steps):
            self.net.forward(Xn)
            dy, loss = self.net.mse_grad(yn)
            self.net.backward(dy)
            self.net.adam(lr=lr)
        return float(loss.item())

    def grad(self, x: np.ndarray):
        """(F_hat(x), dF_hat/dx) from the network's input gradient."""
        xn = torch.from_numpy(((x - self.mx) / self.sx).astype(np.float32)[None]).cuda()
        yhat = self.net.forward(xn)
        dx = self.net.backward(torch.ones(1, device="cuda", dtype=torch.float32),
                               want_dx=True)
        g = dx.cpu().numpy()[0].astype(np.float64) * self.sy / self.sx
        return float(yhat.item()) * self.sy + self.my, g


def surrogate_bfgs(ev: Evaluator, theta0, surrogate: Surrogate, h=1e-3, ftol=1e-6,
                   gtol=1e-4, max_iter=100, f_target: Optional[float] = None,
                   target_rtol: float = 1e-6, train_steps=200,
                   min_archive: Optional[int] = None) -> Trace:
    """BFGS in which, after every exact finite-difference step, the surrogate
    (refitted on all exact pairs so far) proposes the next direction from its
    own gradient.  Proposals are judged only by exact values (Armijo on the
    exact F); a rejected proposal hands over to an exact step.  Convergence is
    decided on exact gradients only: when a surrogate step would stop the run
    (tiny change), an exact gradient is taken at the point first."""
    t0 = time.perf_counter()
    tr = Trace()
    x = np.asarray(theta0, np.float64).copy()
    d = x.shape[0]
    F, g = fd_gradient(ev, x, h)
    g_exact = True
    H = np.eye(d)
    min_archive = min_archive or 3 * (2 * d + 1)

    def log(kind):
        tr.theta.append(x.copy()); tr.f.append(F); tr.exact_evals.append(ev.count)
        tr.wall.append(time.perf_counter() - t0); tr.kind.append(kind)

    def converged(rel=None):
        if f_target is not None:
            return abs(F - f_target) <= target_rtol * abs(f_target)
        if np.max(np.abs(g)) <= gtol:
            return True
        return rel is not None and rel <= ftol

    log("start")
    use_sur = False
    rel = None
    for _ in range(max_iter):
        if g_exact and converged(rel):
            break
        if use_sur and len(ev.archive_f) >= min_archive:
            surrogate.fit(np.asarray(ev.archive_x), np.asarray(ev.archive_f),
                          steps=train_steps)
            _, gs = surrogate.grad(x)
            p = -H @ gs
            if gs @ p < 0:
                a, xn, Fn = _line_search(ev, x, F, gs, p)
                if a is not None and Fn < F:
                    _, gsn = surrogate.grad(xn)
                    H = _bfgs_update(H, xn - x, gsn - gs)
                    rel = abs(Fn - F) / max(1.0, abs(F))
                    x, F, g, g_exact = xn, Fn, gsn, False
                    log("surrogate")
                    if f_target is not None and converged():
                        break
                    # a tiny change is checked by an exact step next
                    use_sur = rel > ftol
                    continue
            use_sur = False   # rejected: take an exact step next
        if not g_exact:
            F, g = fd_gradient(ev, x, h)
            g_exact = True
            if converged():
                break
        p = -H @ g
        if g @ p >= 0:
            H = np.eye(d)
            p = -g
        a, xn, Fn = _line_search(ev, x, F, g, p)
        if a is None:
            break
        Fn2, gn = fd_gradient(ev, xn, h)
        H = _bfgs_update(H, xn - x, gn - g)
        rel = abs(Fn2 - F) / max(1.0, abs(F))
        x, F, g = xn, Fn2, gn
        log("fd")
        use_sur = True
    return tr
