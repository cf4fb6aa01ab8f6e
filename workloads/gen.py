"""Seeded synthetic workloads for the f_obj hot path.

This module only draws data: grid sizes, observation rows (a time step, the
three nodes of one mesh triangle and their barycentric weights), covariates,
responses and hyperparameter vectors.  It holds none of the method's
arithmetic (no precision matrix, no mixing, no likelihood), so that the CPU
oracle and the GPU library can both consume it without sharing any code.

Shapes follow the paper's workloads (a regular spatial mesh of ``nx*nx``
nodes, ``nt`` time steps, ``nv`` response variables, ``nr`` fixed effects
per response, Table 2 of the paper for the model family) at the sizes of the
configurations named below.

Observation rows (one triangle of a uniformly drawn mesh cell):
  * cell (ix, iy) uniform in [0, nx-2]^2;
  * triangle 0 = {(ix,iy), (ix+1,iy), (ix,iy+1)},
    triangle 1 = {(ix+1,iy), (ix,iy+1), (ix+1,iy+1)}, drawn uniformly;
  * weights ~ Dirichlet(1,1,1);
  * time step of row k is k mod nt (exactly m/nt rows per step);
  * covariates iid N(0,1), no intercept.
Node index of grid point (ix, iy) is iy*nx + ix.

Hyperparameter vectors are given in the internal parametrisation that the
library and the oracle both accept:
  univariate  [log kappa, phi, log tau_u, log tau_y]
  trivariate  [log kappa_1..3, phi_1..3, log sigma_1..3, lambda_1..3,
               log tau_y_1..3]
with phi = log((1+rho)/(1-rho)).  A workload of the diffusion-based
(non-separable) space-time model (``model="diffusion"``) puts log gamma_s and
log gamma_t of each process in the slots of log kappa and phi; the other
slots keep their meaning.

A workload with ``likelihood="poisson"`` holds counts instead of Gaussian
responses and its theta has no log tau_y slots.  Its counts are drawn as
Poisson(exp(eta)) with the log rate eta = log(3) + 0.3 s + 0.3 X beta, s
the smooth random space-time signal below at the row's cell and time, beta
iid N(0,1): rates of about 1 to 10, zeros included.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Response:
    """Observation rows of one response variable."""
    t: np.ndarray        # (m,) int32 time step of each row
    nodes: np.ndarray    # (m, 3) int32 node indices (iy*nx + ix)
    w: np.ndarray        # (m, 3) float64 barycentric weights (rows sum to 1)
    X: np.ndarray        # (m, nr) float64 covariates
    y: np.ndarray        # (m,) float64 observed values


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    nt: int
    nv: int
    nr: int
    responses: List[Response]
    theta: np.ndarray            # evaluation point (internal parametrisation)
    theta_prior_mean: np.ndarray  # mean of the Gaussian prior on theta
    theta_prior_sd: float = 1.0
    prior_fixed: float = 1e-3     # precision of each fixed effect
    seed: int = 0
    model: str = "separable"      # or "diffusion" (non-separable)
    likelihood: str = "gaussian"  # or "poisson" (counts)

    @property
    def ns(self) -> int:
        return self.nx * self.nx

    @property
    def b(self) -> int:
        return self.nv * self.ns

    @property
    def a(self) -> int:
        return self.nv * self.nr

    @property
    def N(self) -> int:
        return self.nt * self.b + self.a

    @property
    def m(self) -> int:
        return int(sum(r.y.shape[0] for r in self.responses))

    @property
    def dim_theta(self) -> int:
        base = 4 if self.nv == 1 else 4 * self.nv + self.nv * (self.nv - 1) // 2
        return base - self.nv if self.likelihood == "poisson" else base


def _phi(rho: float) -> float:
    return math.log((1.0 + rho) / (1.0 - rho))


def _draw_rows(rng: np.random.Generator, nx: int, nt: int, m: int, nr: int):
    cells = rng.integers(0, nx - 1, size=(m, 2))          # (ix, iy)
    tri = rng.integers(0, 2, size=m)
    w = rng.dirichlet(np.ones(3), size=m)
    X = rng.standard_normal((m, nr))
    ix, iy = cells[:, 0], cells[:, 1]
    n00 = iy * nx + ix
    n10 = iy * nx + ix + 1
    n01 = (iy + 1) * nx + ix
    n11 = (iy + 1) * nx + ix + 1
    nodes = np.where(tri[:, None] == 0,
                     np.stack([n00, n10, n01], axis=1),
                     np.stack([n10, n01, n11], axis=1)).astype(np.int32)
    t = (np.arange(m) % nt).astype(np.int32)
    return t, nodes, w, X, cells


def _smooth_signal(rng: np.random.Generator, nx: int, nt: int, cells, t,
                   nfreq: int = 6) -> np.ndarray:
    """A smooth random space-time signal evaluated at cell centres."""
    cx = cells[:, 0] + 0.5
    cy = cells[:, 1] + 0.5
    out = np.zeros(cells.shape[0])
    for _ in range(nfreq):
        fx, fy = rng.uniform(0.2, 2.0, size=2) / nx
        ft = rng.uniform(0.0, 0.3)
        ph = rng.uniform(0, 2 * math.pi)
        amp = rng.standard_normal()
        out += amp * np.cos(2 * math.pi * (fx * cx + fy * cy) + ft * t + ph)
    return out


def _check_model(model: str, likelihood: str = "gaussian") -> None:
    if model not in ("separable", "diffusion"):
        raise ValueError(f"unknown model family {model!r}")
    if likelihood not in ("gaussian", "poisson"):
        raise ValueError(f"unknown likelihood {likelihood!r}")


def _counts(rng: np.random.Generator, nx: int, nt: int, cells, t, X) -> np.ndarray:
    """Poisson counts around a smooth log rate (see the module notes)."""
    beta = rng.standard_normal(X.shape[1])
    eta = math.log(3.0) + 0.3 * _smooth_signal(rng, nx, nt, cells, t) + 0.3 * (X @ beta)
    return rng.poisson(np.exp(eta)).astype(np.float64)


def make_univariate(name: str, nx: int, nt: int, nr: int, m: int, *,
                    kappa: float = 1.0, rho: float = 0.7, tau_u: float = 1.0,
                    tau_y: float = 4.0, seed: int = 0,
                    model: str = "separable", gamma_s: float = 1.0,
                    gamma_t: float = 2.0, likelihood: str = "gaussian") -> Workload:
    """Univariate workload: responses y ~ N(0,1), one observation set (or
    counts, ``likelihood="poisson"``).
    ``model="diffusion"`` takes gamma_s, gamma_t in place of kappa, rho."""
    _check_model(model, likelihood)
    rng = np.random.default_rng(seed)
    t, nodes, w, X, cells = _draw_rows(rng, nx, nt, m, nr)
    if likelihood == "poisson":
        y = _counts(rng, nx, nt, cells, t, X)
    else:
        y = rng.standard_normal(m)
    if model == "diffusion":
        head = [math.log(gamma_s), math.log(gamma_t)]
    else:
        head = [math.log(kappa), _phi(rho)]
    tail = [math.log(tau_y)] if likelihood == "gaussian" else []
    theta = np.array(head + [math.log(tau_u)] + tail)
    return Workload(name=name, nx=nx, nt=nt, nv=1, nr=nr,
                    responses=[Response(t, nodes, w, X, y)],
                    theta=theta, theta_prior_mean=theta.copy(), seed=seed,
                    model=model, likelihood=likelihood)


def make_trivariate(name: str, nx: int, nt: int, nr: int, m_per: int, *,
                    kappa=(0.5, 1.0, 2.0), rho=(0.6, 0.8, 0.9),
                    tau_y=(4.0, 4.0, 4.0), seed: int = 0,
                    nv: int = 3, model: str = "separable",
                    gamma_s=(0.5, 1.0, 2.0),
                    gamma_t=(1.0, 2.0, 4.0),
                    likelihood: str = "gaussian") -> Workload:
    """Coregional workload with nv responses.

    sigma_i = max(|z|, 0.5) and lambda_i ~ N(0,1) play the role of the
    lower-triangular coregionalisation matrix with N(0,1) entries and a
    positive diagonal.  Responses are a smooth random signal at the cell of
    each row, plus covariate effects, plus N(0, 1/tau_y) noise, so that the
    optimum of the objective lies inside the parameter space.
    ``model="diffusion"`` takes gamma_s, gamma_t in place of kappa, rho.
    ``likelihood="poisson"``: counts per response (module notes), no tau_y.
    """
    _check_model(model, likelihood)
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(nv)
    sigma = np.maximum(np.abs(z), 0.5)
    lam = rng.standard_normal(nv * (nv - 1) // 2)
    responses = []
    for j in range(nv):
        t, nodes, w, X, cells = _draw_rows(rng, nx, nt, m_per, nr)
        responses.append([t, nodes, w, X, cells])
    for j in range(nv):
        t, nodes, w, X, cells = responses[j]
        if likelihood == "poisson":
            responses[j] = Response(t, nodes, w, X, _counts(rng, nx, nt, cells, t, X))
            continue
        beta = rng.standard_normal(nr)
        sig = _smooth_signal(rng, nx, nt, cells, t)
        noise = rng.standard_normal(m_per) / math.sqrt(tau_y[j])
        y = sig + X @ beta + noise
        responses[j] = Response(t, nodes, w, X, y)
    if model == "diffusion":
        head = [np.log(np.asarray(gamma_s[:nv], np.float64)),
                np.log(np.asarray(gamma_t[:nv], np.float64))]
    else:
        head = [np.log(np.asarray(kappa[:nv])),
                np.array([_phi(r) for r in rho[:nv]])]
    tail = [np.log(np.asarray(tau_y[:nv]))] if likelihood == "gaussian" else []
    theta = np.concatenate(head + [np.log(sigma), lam] + tail)
    return Workload(name=name, nx=nx, nt=nt, nv=nv, nr=nr,
                    responses=responses, theta=theta,
                    theta_prior_mean=theta.copy(), seed=seed, model=model,
                    likelihood=likelihood)


# --- the named configurations ------------------------------------------------

def config0(seed: int = 0) -> Workload:
    """Tiny univariate: 10x10 grid, nt=10, nr=2, m=400 (N=1002)."""
    return make_univariate("c0_univariate_10x10_nt10", 10, 10, 2, 400,
                           seed=seed)


def _suffix(model: str) -> str:
    return "" if model == "separable" else "_" + model


def config1(seed: int = 0, model: str = "separable",
            likelihood: str = "gaussian") -> Workload:
    """Production univariate: 45x45 grid (b=2025), nt=100, nr=4, m=200000
    (counts with ``likelihood="poisson"``)."""
    name = "c1_univariate_45x45_nt100" + _suffix(model)
    if likelihood != "gaussian":
        name += "_" + likelihood
    return make_univariate(name, 45, 100, 4, 200_000, seed=seed, model=model,
                           likelihood=likelihood)


def config2(seed: int = 0, model: str = "separable",
            likelihood: str = "gaussian") -> Workload:
    """Trivariate coregional: 30x30 grid (b=2700), nt=48, nr=2 (a=6),
    m = 3 x 48 x 900 (counts with ``likelihood="poisson"``)."""
    name = "c2_trivariate_30x30_nt48" + _suffix(model)
    if likelihood != "gaussian":
        name += "_" + likelihood
    return make_trivariate(name, 30, 48, 2, 48 * 900, seed=seed, model=model,
                           likelihood=likelihood)


def scaled(name: str, nx: int, nt: int, nv: int, nr: int, m_per: int,
           seed: int = 0, model: str = "separable",
           likelihood: str = "gaussian") -> Workload:
    """Same generator at other sizes (parity cases, edge cases)."""
    if nv == 1:
        return make_univariate(name, nx, nt, nr, m_per, seed=seed, model=model,
                               likelihood=likelihood)
    return make_trivariate(name, nx, nt, nr, m_per, seed=seed, nv=nv,
                           model=model, likelihood=likelihood)


def uneven_instance(k: int) -> Workload:
    """Instance k of the 64-instance uneven batch (nv, ns, nt, nr mix)."""
    nv = [1, 3][k % 2]
    nx = [20, 30, 45][(k // 2) % 3]          # ns in {400, 900, 2025}
    nt = [12, 24, 48, 100][(k // 6) % 4]
    nb = [2, 6][(k // 24) % 2]               # fixed effects in total
    nr = max(1, nb // nv)
    m_per = nt * nx * nx // 2
    return scaled(f"uneven_{k}", nx, nt, nv, nr, m_per, seed=k)


def random_theta_near(theta: np.ndarray, scale: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(1000 + seed)
    return theta + scale * rng.standard_normal(theta.shape[0])
