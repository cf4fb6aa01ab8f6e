"""Mode search over theta (Eq. 9) on top of the batched evaluator.

Two drivers minimise F(theta) = -f_obj(theta):

* ``fd_bfgs``: BFGS with the central-difference gradient of Eq. 10.  The
  2*dim+1 stencil points of one gradient are one batched evaluation pass;
  the line search evaluates a short ladder of step lengths (1, 1/2, 1/4,
  1/8, then the next four if none qualifies, ...) as one small batched pass
  and keeps the longest step with sufficient (Armijo) decrease.  The search
  direction is capped at length ``max_step`` (theta holds log-scale
  parameters), the initial inverse Hessian is rescaled by y^T s / y^T y
  before the first update, and a failed line search is retried once along
  the steepest-descent direction.
* ``surrogate_bfgs``: the same exact steps, but after each one a learned
  surrogate -- the GPU MLP, trained online (warm-started) on every exact
  (theta, F) pair so far -- supplies the gradient for up to ``max_sur``
  further quasi-Newton steps, each costing one line-search pass instead of a
  finite-difference gradient.  Every proposed point is evaluated exactly and
  accepted only on exact values (Armijo along the surrogate's slope); the
  surrogate streak ends as soon as the exact decrease falls below ``eta``
  times the decrease the surrogate predicted.  The BFGS matrix is updated
  only from exact gradients (one secant pair per finite-difference pass) and
  convergence is decided on exact gradients only.

Host-side logic only (vectors of length dim theta); every f_obj value comes
from the library's kernels.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, List, Optional

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
    H: Optional[np.ndarray] = None  # final inverse-Hessian estimate (BFGS drivers)


class Evaluator:
    """Batched exact evaluation of F = -f_obj on one model: a workspace of
    `batch` instances for gradient stencils and one of `ntrial` instances for
    line searches."""

    def __init__(self, model: "D.Model", batch: int, graph: bool = True, ntrial: int = 4,
                 warm_start: Optional[bool] = None, mixed: bool = False):
        self.model = model
        self.mixed = mixed
        self.B = batch
        self.ntrial = ntrial
        # warm_start (Poisson likelihood; the default for it): each instance's
        # inner Newton search starts from its mode of the previous pass, which
        # the nearby points of consecutive gradients and line searches reuse
        if warm_start is None:
            warm_start = getattr(model, "likelihood", "gaussian") == "poisson"
        self.ws = D.Workspace([model] * batch, graph=graph, warm_start=warm_start,
                              mixed=mixed)
        self.ws_ls = D.Workspace([model] * ntrial, graph=graph, warm_start=warm_start,
                                 mixed=mixed)
        self.dim = model.dim_theta
        self.count = 0
        self.archive_x: List[np.ndarray] = []
        self.archive_f: List[float] = []

    def __call__(self, thetas: np.ndarray) -> np.ndarray:
        thetas = np.atleast_2d(np.asarray(thetas, np.float64))
        n = thetas.shape[0]
        if n > self.B:
            return np.concatenate([self(thetas[i:i + self.B]) for i in range(0, n, self.B)])
        ws, size = (self.ws_ls, self.ntrial) if n <= self.ntrial else (self.ws, self.B)
        if n < size:  # pad with copies of the first point (not counted)
            thetas_p = np.concatenate([thetas, np.repeat(thetas[:1], size - n, axis=0)])
        else:
            thetas_p = thetas
        f, _, _ = ws.fobj(thetas_p)
        vals = -f.cpu().numpy()[:n]
        self.count += n
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


def _capped(p, max_step):
    nrm = float(np.linalg.norm(p))
    return p * (max_step / nrm) if nrm > max_step else p


def _line_search(ev: Evaluator, theta, F0, g, p, c1=1e-4, max_passes=4):
    """Evaluate theta + alpha p for alpha = 1, 1/2, ... (ev.ntrial per pass);
    return the longest step with F <= F0 + c1 alpha g.p, else
    (None, None, None)."""
    slope = float(g @ p)
    for k in range(max_passes):
        alphas = 0.5 ** (k * ev.ntrial + np.arange(ev.ntrial))
        vals = ev(theta[None, :] + alphas[:, None] * p[None, :])
        for a, v in zip(alphas, vals):
            if np.isfinite(v) and v <= F0 + c1 * a * slope:
                return a, theta + a * p, v
    return None, None, None


def _bfgs_update(H, s, y, first=False):
    ys = float(y @ s)
    if not (ys > 1e-12 and np.isfinite(ys) and np.all(np.isfinite(y))):
        return H
    if first:
        H = (ys / float(y @ y)) * np.eye(H.shape[0])
    r = 1.0 / ys
    I = np.eye(H.shape[0])
    return (I - r * np.outer(s, y)) @ H @ (I - r * np.outer(y, s)) + r * np.outer(s, s)


def _exact_step(ev, x, F, g, H, max_step):
    """Quasi-Newton step with the capped direction; one retry along the
    steepest-descent direction.  Returns (alpha, x_new, F_new, H)."""
    p = -H @ g
    if g @ p >= 0:
        H = np.eye(x.shape[0])
        p = -g
    a, xn, Fn = _line_search(ev, x, F, g, _capped(p, max_step))
    if a is None:
        H = np.eye(x.shape[0])
        a, xn, Fn = _line_search(ev, x, F, g, _capped(-g, max_step))
    return a, xn, Fn, H


def fd_bfgs(ev: Evaluator, theta0, h=1e-3, ftol=1e-6, gtol=1e-4, max_iter=100,
            f_target: Optional[float] = None, target_rtol: float = 1e-6,
            max_step: float = 1.0, f_check: Optional[Callable[[np.ndarray], float]] = None,
            count: Optional[Callable[[], int]] = None, kind: str = "fd",
            H0: Optional[np.ndarray] = None, check_band: float = math.inf,
            min_progress: float = 0.0) -> Trace:
    """f_check (optional): the value the target test uses at each iterate
    instead of ev's (an FP64 evaluation when ev is mixed precision), called
    only where ev's value lies within target_rtol |f_target| + check_band of
    the target; count: the evaluation counter the trace records (default
    ev.count); H0: the starting inverse-Hessian estimate (default I, scaled
    at the first update), returned updated as the trace's H; min_progress:
    stop once an iteration lowers F by less than this."""
    t0 = time.perf_counter()
    tr = Trace()
    x = np.asarray(theta0, np.float64).copy()
    F, g = fd_gradient(ev, x, h)
    H = np.eye(x.shape[0]) if H0 is None else np.array(H0, np.float64)
    first = H0 is None
    count = count or (lambda: ev.count)

    def log(k):
        tr.theta.append(x.copy()); tr.f.append(F); tr.exact_evals.append(count())
        tr.wall.append(time.perf_counter() - t0); tr.kind.append(k)

    log("start")
    for _ in range(max_iter):
        if not (np.isfinite(F) and np.all(np.isfinite(g))):
            break  # a stencil point without a value (not positive definite there)
        if f_target is not None:
            tol = target_rtol * abs(f_target)
            if f_check is None:
                Fc = F
            elif abs(F - f_target) <= tol + check_band:
                Fc = f_check(x)
            else:
                Fc = math.inf
            if abs(Fc - f_target) <= tol:
                break
        if np.max(np.abs(g)) <= gtol:
            break
        a, xn, Fn, H = _exact_step(ev, x, F, g, H, max_step)
        if a is None:
            break
        Fn2, gn = fd_gradient(ev, xn, h)
        H = _bfgs_update(H, xn - x, gn - g, first)
        first = False
        rel = abs(Fn2 - F) / max(1.0, abs(F))
        gain = F - Fn2
        x, F, g = xn, Fn2, gn
        log(kind)
        if f_target is None and rel <= ftol:
            break
        if gain < min_progress:
            break
    tr.H = H
    return tr


def mixed_fd_bfgs(ev: Evaluator, ev64: Evaluator, theta0, h=1e-3, ftol=1e-6, gtol=1e-4,
                  max_iter=100, f_target: Optional[float] = None,
                  target_rtol: float = 1e-6, max_step: float = 1.0,
                  h_mixed: Optional[float] = None, check_band: float = 1e-5,
                  stall_rtol: float = 1e-6) -> Trace:
    """FD-BFGS on the mixed-precision evaluator `ev`, then FD-BFGS on the
    FP64 evaluator `ev64` from the point where the mixed search stops (a
    failed line search or ftol/gtol on its values: the floor its FP32
    rounding puts under the finite differences), starting from the mixed
    phase's inverse-Hessian estimate.

    The mixed phase differences with h_mixed (default 30 h): the FP32
    rounding of the off-diagonal blocks perturbs f by an amount that does not
    vary smoothly with theta, so central differences over h would be mostly
    that noise; over 30 h the noise term shrinks 30-fold while the
    truncation error stays small far from the optimum, which is where the
    mixed phase works.  With f_target the target is tested on FP64 values,
    one ev64 evaluation per mixed iterate whose mixed value is within
    target_rtol |f_target| + check_band |f_target| of the target.  The mixed
    phase also stops once an iteration gains less than stall_rtol |F| (gains
    below the FP32 perturbation are not to be trusted).  The
    trace's f are the evaluator's own values (mixed in the first phase, kind
    'mixed'; FP64 in the second, kind 'fd'); exact_evals counts both
    evaluators."""
    total = lambda: ev.count + ev64.count
    check = (lambda x: float(ev64(x[None])[0])) if f_target is not None else None
    hm = 30.0 * h if h_mixed is None else h_mixed
    band = check_band * abs(f_target) if f_target is not None else math.inf
    t1 = fd_bfgs(ev, theta0, h=hm, ftol=ftol, gtol=gtol, max_iter=max_iter,
                 f_target=f_target, target_rtol=target_rtol, max_step=max_step,
                 f_check=check, count=total, kind="mixed", check_band=band,
                 min_progress=stall_rtol * abs(f_target if f_target is not None
                                                else ev(np.asarray(theta0)[None])[0]))
    x1 = t1.theta[-1]
    if f_target is not None and abs(check(x1) - f_target) <= target_rtol * abs(f_target):
        return t1
    # no accepted mixed step: no curvature yet
    H1 = t1.H if len(t1.f) > 1 and np.all(np.isfinite(t1.H)) else None
    t2 = fd_bfgs(ev64, x1, h=h, ftol=ftol, gtol=gtol, max_iter=max_iter,
                 f_target=f_target, target_rtol=target_rtol, max_step=max_step,
                 count=total, H0=H1)
    off = t1.wall[-1]
    for i in range(len(t2.f)):
        t1.theta.append(t2.theta[i]); t1.f.append(t2.f[i])
        t1.exact_evals.append(t2.exact_evals[i]); t1.wall.append(off + t2.wall[i])
        t1.kind.append("fp64-start" if i == 0 else t2.kind[i])
    t1.H = t2.H
    return t1


class Surrogate:
    """Online MLP model of F over theta, trained with the GPU kernels.  The
    input centring/scaling and output standardisation are fixed at the first
    fit, so later fits continue from the current weights (online training)."""

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
        self.fitted = False

    def fit(self, X: np.ndarray, y: np.ndarray, steps=200, lr=2e-3):
        if not self.fitted:
            self.mx = X.mean(axis=0)
            self.sx = X.std(axis=0) + 1e-2
            self.my = float(y.mean())
            self.sy = float(y.std() + 1e-12)
            self.fitted = True
        if X.shape[0] > self.net.max_batch:  # the most recent pairs
            X, y = X[-self.net.max_batch:], y[-self.net.max_batch:]
        Xn = torch.from_numpy(((X - self.mx) / self.sx).astype(np.float32)).cuda()
        yn = torch.from_numpy(((y - self.my) / self.sy).astype(np.float32)).cuda()
        loss = None
        for _ in range(steps):
            self.net.forward(Xn)
            dy, loss = self.net.mse_grad(yn)
            self.net.backward(dy)
            self.net.adam(lr=lr)
        return float(loss.item()) if loss is not None else float("nan")

    def predict(self, x: np.ndarray) -> float:
        xn = torch.from_numpy(((x - self.mx) / self.sx).astype(np.float32)[None]).cuda()
        return float(self.net.forward(xn).item()) * self.sy + self.my

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
                   target_rtol: float = 1e-6, train_steps=100,
                   min_archive: Optional[int] = None, max_step: float = 1.0,
                   max_sur: int = 3, eta: float = 0.25) -> Trace:
    t0 = time.perf_counter()
    tr = Trace()
    x = np.asarray(theta0, np.float64).copy()
    d = x.shape[0]
    F, g = fd_gradient(ev, x, h)
    H = np.eye(d)
    first = True
    min_archive = min_archive or 2 * (2 * d + 1)

    def log(kind, xx, FF):
        tr.theta.append(xx.copy()); tr.f.append(FF); tr.exact_evals.append(ev.count)
        tr.wall.append(time.perf_counter() - t0); tr.kind.append(kind)

    def reached(FF):
        return f_target is not None and abs(FF - f_target) <= target_rtol * abs(f_target)

    log("start", x, F)
    for _ in range(max_iter):
        if reached(F) or np.max(np.abs(g)) <= gtol:
            break
        a, xs, Fs, H = _exact_step(ev, x, F, g, H, max_step)
        if a is None:
            break
        log("exact-step", xs, Fs)
        if len(ev.archive_f) >= min_archive and not reached(Fs):
            surrogate.fit(np.asarray(ev.archive_x), np.asarray(ev.archive_f),
                          steps=train_steps)
            for _ in range(max_sur):
                Fh, gs = surrogate.grad(xs)
                p = _capped(-H @ gs, max_step)
                if gs @ p >= 0:
                    break
                a2, x2, F2 = _line_search(ev, xs, Fs, gs, p, max_passes=1)
                if a2 is None:
                    break
                pred = Fh - surrogate.predict(x2)
                actual = Fs - F2
                xs, Fs = x2, F2
                log("surrogate", xs, Fs)
                if pred <= 0 or actual < eta * pred or reached(Fs):
                    break
        Fn2, gn = fd_gradient(ev, xs, h)
        H = _bfgs_update(H, xs - x, gn - g, first)
        first = False
        rel = abs(Fn2 - F) / max(1.0, abs(F))
        x, F, g = xs, Fn2, gn
        log("fd", x, F)
        if f_target is None and rel <= ftol:
            break
    return tr
