"""CPU FP64 oracle -- model assembly.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in
``oracle/``; the GPU library never does.  It shares no code with the GPU path.

Plain, slow, obviously-correct construction of the prior precision Q_p and
the conditional precision Q_c of the paper's spatio-temporal (optionally
coregional) latent Gaussian model, as general scipy sparse matrices in
*model order* (response-major, then time, then space; fixed effects last):

    z_j(t, s)  -> j*(nt*ns) + t*ns + s
    beta_j(r)  -> nv*nt*ns + j*nr + r

Readings of points the paper leaves open (grid spacing h = 1; Neumann
5-point stiffness; lumped mass; AR1 with unit marginal variance; Kronecker
order time-outer; fixed effects not mixed by Lambda; Gaussian prior on
theta; the form of the non-separable diffusion-based model) are stated on
each function.

Two model families: ``wl.model == "separable"`` (AR1 in time times the
Matern SPDE precision in space) and ``"diffusion"``, the non-separable
space-time model written as a sum of Kronecker products of temporal and
spatial FEM matrices (Section IV-B, multivariate model formulation, which builds every
univariate precision that way).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


# --- hyperparameters -----------------------------------------------------------

def n_lambda(nv: int) -> int:
    return nv * (nv - 1) // 2


LIKELIHOODS = ("gaussian", "poisson")


def theta_dim(nv: int, likelihood: str = "gaussian") -> int:
    """Gaussian responses carry one noise precision each; Poisson responses
    have no likelihood hyperparameter."""
    base = 4 if nv == 1 else 4 * nv + n_lambda(nv)
    return base - nv if likelihood == "poisson" else base


def theta_to_params(theta, nv: int, model: str = "separable",
                    likelihood: str = "gaussian") -> dict:
    """Internal theta -> model parameters.

    Univariate: [log kappa, phi, log tau_u, log tau_y].
    Coregional: [log kappa_i, phi_i, log sigma_i, lambda_k, log tau_y_j].
    A Poisson likelihood drops the trailing log tau_y slots (tau_y = None).
    rho = tanh(phi/2) inverts phi = log((1+rho)/(1-rho)), which keeps the AR1
    coefficient inside (-1, 1) for every real phi.  Optimisation is
    unconstrained over theta (Eq. 9).

    The diffusion-based model reads the first two slots of each process as
    log gamma_s and log gamma_t (spatial and temporal rate of the diffusion
    operator, see ``diffusion_precision``); the remaining slots keep their
    meaning, so the dimension of theta does not change.
    """
    th = np.asarray(theta, dtype=np.float64)
    if likelihood not in LIKELIHOODS:
        raise ValueError(f"unknown likelihood {likelihood!r}")
    assert th.shape == (theta_dim(nv, likelihood),)
    if model not in ("separable", "diffusion"):
        raise ValueError(f"unknown model family {model!r}")
    gauss = likelihood == "gaussian"
    if nv == 1:
        out = dict(sigma=np.array([1.0 / math.sqrt(math.exp(th[2]))]),
                   lam=np.zeros(0), tau_y=np.exp(th[3:4]) if gauss else None,
                   tau_u=math.exp(th[2]))
        head = (th[0:1], th[1:2])
    else:
        k = 2 * nv
        sigma = np.exp(th[k:k + nv]); k += nv
        lam = th[k:k + n_lambda(nv)].copy(); k += n_lambda(nv)
        tau_y = np.exp(th[k:k + nv]) if gauss else None
        out = dict(sigma=sigma, lam=lam, tau_y=tau_y, tau_u=None)
        head = (th[0:nv], th[nv:2 * nv])
    if model == "diffusion":
        out.update(gamma_s=np.exp(head[0]), gamma_t=np.exp(head[1]))
    else:
        out.update(kappa=np.exp(head[0]), rho=np.tanh(head[1] / 2))
    return out


def log_prior_theta(theta, mean, sd: float) -> float:
    """log p(theta) of Eq. 7/8.  The paper does not fix this prior; read as
    independent Gaussians N(mean_k, sd^2) on the internal parameters,
    normalising constant included."""
    th = np.asarray(theta, np.float64)
    mu = np.asarray(mean, np.float64)
    d = th.shape[0]
    return float(-0.5 * d * math.log(2 * math.pi * sd * sd)
                 - 0.5 * np.sum((th - mu) ** 2) / (sd * sd))


# --- spatial SPDE precision (FEM on a regular grid) ------------------------------

def node_index(ix, iy, nx):
    return iy * nx + ix


def stiffness_G(nx: int) -> sp.csr_matrix:
    """Stiffness G of the FEM discretisation of the SPDE on an nx*nx grid
    with unit spacing and natural (Neumann) boundary: the 5-point graph
    Laplacian -- degree on the diagonal, -1 for each grid neighbour."""
    ns = nx * nx
    rows, cols = [], []
    for iy in range(nx):
        for ix in range(nx):
            s = node_index(ix, iy, nx)
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                jx, jy = ix + dx, iy + dy
                if 0 <= jx < nx and 0 <= jy < nx:
                    rows.append(s)
                    cols.append(node_index(jx, jy, nx))
    A = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(ns, ns))
    deg = np.asarray(A.sum(axis=1)).ravel()
    return (sp.diags(deg) - A).tocsr()


def mass_C(nx: int) -> sp.csr_matrix:
    """Lumped mass matrix C = h^2 I with h = 1."""
    return sp.identity(nx * nx, format="csr")


def spatial_precision(nx: int, kappa: float) -> sp.csr_matrix:
    """Q_s(kappa) = kappa^4 C + 2 kappa^2 G + G C^{-1} G, the SPDE precision of
    the Matern-type field (Section II-A, SPDE approach)."""
    C = mass_C(nx)
    G = stiffness_G(nx)
    Cinv = sp.diags(1.0 / C.diagonal())
    return (kappa ** 4 * C + 2 * kappa ** 2 * G + G @ Cinv @ G).tocsr()


# --- temporal AR1 precision -------------------------------------------------------

def ar1_precision(nt: int, rho: float) -> sp.csr_matrix:
    """Precision of a stationary AR1 process x_t = rho x_{t-1} + e_t scaled to
    unit marginal variance: (1-rho^2)^{-1} tridiag(-rho; [1, 1+rho^2, ...,
    1+rho^2, 1]; -rho).  For nt = 1 it is the 1x1 matrix [1]."""
    if nt == 1:
        return sp.csr_matrix(np.ones((1, 1)))
    d = np.full(nt, 1.0 + rho * rho)
    d[0] = d[-1] = 1.0
    off = np.full(nt - 1, -rho)
    T = sp.diags([off, d, off], [-1, 0, 1]) / (1.0 - rho * rho)
    return T.tocsr()


def spacetime_precision(nx: int, nt: int, kappa: float, rho: float):
    """Separable space-time precision T (x) Q_s with time ordered outermost
    (variables ordered sequentially over time, which gives the block
    tridiagonal pattern of Section II-A)."""
    return sp.kron(ar1_precision(nt, rho), spatial_precision(nx, kappa),
                   format="csr")


# --- non-separable diffusion-based space-time precision ----------------------------

def temporal_fem(nt: int):
    """Temporal FEM matrices of piecewise-linear elements on the time nodes
    0, 1, ..., nt-1 (unit spacing):

      M0  lumped mass: the integral of each hat function, 1/2 at the two end
          nodes and 1 inside;
      M1  boundary matrix: 1/2 at the two end nodes, 0 elsewhere;
      M2  stiffness: the integrals of products of hat-function derivatives,
          tridiag(-1; [1, 2, ..., 2, 1]; -1).

    Needs nt >= 2 (one node spans no interval)."""
    if nt < 2:
        raise ValueError("the diffusion-based model needs nt >= 2")
    m0 = np.ones(nt)
    m0[0] = m0[-1] = 0.5
    m1 = np.zeros(nt)
    m1[0] = m1[-1] = 0.5
    d2 = np.full(nt, 2.0)
    d2[0] = d2[-1] = 1.0
    off = -np.ones(nt - 1)
    return (sp.diags(m0).tocsr(), sp.diags(m1).tocsr(),
            sp.diags([off, d2, off], [-1, 0, 1]).tocsr())


def spatial_operator_powers(nx: int, gamma_s: float):
    """K_k, k = 1, 2, 3: the FEM matrices of L^k for L = gamma_s^2 - Laplace,
    K_1 = gamma_s^2 C + G and K_{k+1} = K_1 C^{-1} K_k."""
    C = mass_C(nx)
    G = stiffness_G(nx)
    Cinv = sp.diags(1.0 / C.diagonal())
    K1 = (gamma_s ** 2 * C + G).tocsr()
    K2 = (K1 @ Cinv @ K1).tocsr()
    K3 = (K1 @ Cinv @ K2).tocsr()
    return K1, K2, K3


def diffusion_precision(nx: int, nt: int, gamma_s: float, gamma_t: float):
    """Non-separable space-time precision as a sum of Kronecker products of
    temporal and spatial FEM matrices, time outermost (Section IV-B,
    multivariate models, citing the diffusion-based family of Lindgren et
    al.).  The paper gives no formula; read as the critical diffusion model
    with one time derivative, a second-order spatial operator and a
    first-order smoothing of the driving noise:

        Q = M0 (x) K_3 + 2 gamma_t M1 (x) K_2 + gamma_t^2 M2 (x) K_1,

    the discretised quadratic form of (gamma_t d/dt + L) x with noise
    precision L, the boundary term of the time integral taken with a plus
    sign at both ends (stationary start).  The overall scale is the process
    scale of the surrounding model (tau_u, or sigma_i through Lambda)."""
    M0, M1, M2 = temporal_fem(nt)
    K1, K2, K3 = spatial_operator_powers(nx, gamma_s)
    Q = (sp.kron(M0, K3) + 2.0 * gamma_t * sp.kron(M1, K2)
         + gamma_t ** 2 * sp.kron(M2, K1))
    return Q.tocsr()


def process_precision(wl, p: dict, i: int):
    """Precision of univariate process i (unit process scale)."""
    if getattr(wl, "model", "separable") == "diffusion":
        return diffusion_precision(wl.nx, wl.nt, p["gamma_s"][i],
                                   p["gamma_t"][i])
    return spacetime_precision(wl.nx, wl.nt, p["kappa"][i], p["rho"][i])


# --- coregionalisation (Eq. 5, 6, 11) ------------------------------------------------

def coregionalisation_matrix(sigma, lam) -> np.ndarray:
    """The nv x nv matrix Lambda of Eq. 5 (written there for nv = 3):
       [[s1, 0, 0], [l1 s1, s2, 0], [(l3 + l1 l2) s1, l2 s2, s3]].
    nv = 2 keeps its leading 2x2 block; nv = 1 is [s1]."""
    nv = len(sigma)
    L = np.zeros((nv, nv))
    s = sigma
    if nv >= 1:
        L[0, 0] = s[0]
    if nv >= 2:
        L[1, 0] = lam[0] * s[0]
        L[1, 1] = s[1]
    if nv >= 3:
        L[2, 0] = (lam[2] + lam[0] * lam[1]) * s[0]
        L[2, 1] = lam[1] * s[1]
        L[2, 2] = s[2]
    if nv > 3:
        raise ValueError("nv > 3 is not defined by the paper's Eq. 5")
    return L


def mixing_weights(sigma, lam) -> np.ndarray:
    """M[i, j, k] = (Lambda^{-1})_{ij} (Lambda^{-1})_{ik}: the weight of the
    univariate precision Q^i in block (j, k) of the joint precision
    Lambda^{-T} blockdiag(Q^i) Lambda^{-1} (Eq. 6 inverted, giving Eq. 11)."""
    Li = np.linalg.inv(coregionalisation_matrix(sigma, lam))
    return np.einsum("ij,ik->ijk", Li, Li)


# --- the latent model ------------------------------------------------------------------

def model_family(wl) -> str:
    return getattr(wl, "model", "separable")


def likelihood_family(wl) -> str:
    return getattr(wl, "likelihood", "gaussian")


def prior_precision(wl, theta) -> sp.csr_matrix:
    """Q_p(theta) in model order.

    nv = 1: tau_u (T (x) Q_s), bordered by prior_fixed * I for the fixed
    effects (Eq. 1 with x extended by the fixed effects, Section II-A).
    nv > 1: the joint precision of Eq. 11 built from the univariate
    T^i (x) Q_s^i (each with its own kappa_i, rho_i), bordered likewise.
    The fixed effects are not mixed by Lambda.  The diffusion-based family
    puts ``diffusion_precision`` in place of T (x) Q_s.
    """
    nv, nx, nt = wl.nv, wl.nx, wl.nt
    p = theta_to_params(theta, nv, model_family(wl), likelihood_family(wl))
    nst = nx * nx * nt
    if nv == 1:
        Qz = p["tau_u"] * process_precision(wl, p, 0)
    else:
        Qi = [process_precision(wl, p, i) for i in range(nv)]
        M = mixing_weights(p["sigma"], p["lam"])
        blocks = [[None] * nv for _ in range(nv)]
        for j in range(nv):
            for k in range(nv):
                acc = sp.csr_matrix((nst, nst))
                for i in range(nv):
                    if M[i, j, k] != 0.0:
                        acc = acc + M[i, j, k] * Qi[i]
                blocks[j][k] = acc
        Qz = sp.bmat(blocks, format="csr")
    a = nv * wl.nr
    Qf = wl.prior_fixed * sp.identity(a, format="csr")
    return sp.block_diag([Qz, Qf], format="csr")


def design_matrix(wl) -> sp.csr_matrix:
    """A of Eq. 2 in model order (rows: responses stacked): each row holds the
    three barycentric weights of its triangle at its time step on the field of
    its own response, and its covariates on that response's fixed effects."""
    nv, nr, ns, nt = wl.nv, wl.nr, wl.ns, wl.nt
    nst = ns * nt
    N = nv * nst + nv * nr
    rows, cols, vals = [], [], []
    r0 = 0
    for j, resp in enumerate(wl.responses):
        m = resp.y.shape[0]
        ridx = r0 + np.arange(m)
        for q in range(3):
            rows.append(ridx)
            cols.append(j * nst + resp.t.astype(np.int64) * ns
                        + resp.nodes[:, q])
            vals.append(resp.w[:, q])
        for r in range(nr):
            rows.append(ridx)
            cols.append(np.full(m, nv * nst + j * nr + r))
            vals.append(resp.X[:, r])
        r0 += m
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(r0, N))


def noise_precision(wl, theta) -> np.ndarray:
    """Diagonal of D(theta): the Gaussian likelihood's negative Hessian, i.e.
    tau_y_j for every row of response j (Eq. 4).  Gaussian responses only:
    for other likelihoods D depends on x (see ``oracle.laplace``)."""
    if likelihood_family(wl) != "gaussian":
        raise ValueError("D(theta) alone is defined for Gaussian responses only")
    p = theta_to_params(theta, wl.nv, model_family(wl))
    return np.concatenate([np.full(r.y.shape[0], p["tau_y"][j])
                           for j, r in enumerate(wl.responses)])


def observations(wl) -> np.ndarray:
    return np.concatenate([r.y for r in wl.responses])


def conditional_precision(wl, theta, Qp=None, A=None) -> sp.csr_matrix:
    """Q_c = Q_p + A^T D A (Eq. 4)."""
    if Qp is None:
        Qp = prior_precision(wl, theta)
    if A is None:
        A = design_matrix(wl)
    d = noise_precision(wl, theta)
    return (Qp + (A.T @ sp.diags(d) @ A)).tocsr()


# --- block-tridiagonal-with-arrowhead order ------------------------------------------

def bta_permutation(nv: int, ns: int, nt: int, nr: int) -> np.ndarray:
    """perm[k] = model-order index of the variable at BTA position k.

    BTA order (Section IV-B, permutation): all variables of time step 0 first
    (response by response, each in spatial order), then time step 1, ...,
    with all fixed effects gathered at the end."""
    b = nv * ns
    nst = ns * nt
    perm = np.empty(nt * b + nv * nr, dtype=np.int64)
    k = 0
    for t in range(nt):
        for j in range(nv):
            perm[k:k + ns] = j * nst + t * ns + np.arange(ns)
            k += ns
    perm[k:] = nv * nst + np.arange(nv * nr)
    return perm
