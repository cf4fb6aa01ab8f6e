"""Pins of the CPU oracle against facts that do not come from the oracle.

Each check is chosen so that a plausible slip in the oracle (a dropped term, a
wrong coefficient or sign, a transposed operand, a wrong index map) fails:
closed-form spectra of the FEM and AR1 operators, the Kronecker log-determinant,
the paper's two printed forms of the coregional precision (Eq. 6 vs Eq. 11),
the Gaussian marginal likelihood written without Q_c, the x-invariance of
Eq. 8 for Gaussian data, the dimensions printed in Table 2, and two
independent factorisation routes.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import model as M
from oracle import fobj as F
from oracle.linalg import DenseSPD, BandedSPD

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---- closed forms (written from the spectral theory, not from the oracle) ----

def dct_eigs(nx):
    """Eigenvalues of the Neumann 5-point path Laplacian on nx points."""
    k = np.arange(nx)
    return 2.0 - 2.0 * np.cos(np.pi * k / nx)


def dct_basis(nx):
    """Orthonormal DCT-II eigenvectors of the Neumann path Laplacian."""
    i = np.arange(nx)[:, None]
    k = np.arange(nx)[None, :]
    V = np.cos(np.pi * k * (i + 0.5) / nx) * math.sqrt(2.0 / nx)
    V[:, 0] = 1.0 / math.sqrt(nx)
    return V


def qs_logdet_closed(nx, kappa):
    lam = dct_eigs(nx)
    ev = (kappa ** 2 + lam[:, None] + lam[None, :]) ** 2
    return float(np.sum(np.log(ev)))


def qs_invdiag_closed(nx, kappa):
    lam = dct_eigs(nx)
    V = dct_basis(nx)
    ev = (kappa ** 2 + lam[:, None] + lam[None, :]) ** 2  # (kx, ky)
    # node s = iy*nx + ix; eigvec (kx, ky) = V[ix,kx] V[iy,ky]
    V2 = V * V
    d = np.einsum("xk,yl,kl->yx", V2, V2, 1.0 / ev)
    return d.ravel()


def ar1_logdet_closed(nt, rho):
    return -(nt - 1) * math.log(1.0 - rho * rho)


# ---- pins -----------------------------------------------------------------------

@pytest.mark.parametrize("nx,kappa", [(5, 1.0), (7, 0.5), (8, 2.0)])
def test_spatial_precision_spectrum(nx, kappa):
    Qs = M.spatial_precision(nx, kappa).toarray()
    sign, ld = np.linalg.slogdet(Qs)
    assert sign > 0
    assert abs(ld - qs_logdet_closed(nx, kappa)) < 1e-10 * abs(ld)
    inv = np.diag(np.linalg.inv(Qs))
    np.testing.assert_allclose(inv, qs_invdiag_closed(nx, kappa), rtol=1e-11)
    # the three FEM pieces separately: G is a graph Laplacian (rows sum to 0)
    G = M.stiffness_G(nx)
    assert np.abs(np.asarray(G.sum(axis=1))).max() == 0.0
    ev = np.sort(np.linalg.eigvalsh(G.toarray()))
    lam = dct_eigs(nx)
    np.testing.assert_allclose(ev, np.sort((lam[:, None] + lam[None, :]).ravel()),
                               atol=1e-12)


@pytest.mark.parametrize("nt,rho", [(1, 0.3), (2, 0.5), (9, 0.7), (12, -0.9)])
def test_ar1_closed_forms(nt, rho):
    T = M.ar1_precision(nt, rho).toarray()
    sign, ld = np.linalg.slogdet(T)
    assert sign > 0
    assert abs(ld - ar1_logdet_closed(nt, rho)) < 1e-12 * max(1, abs(ld))
    i = np.arange(nt)
    cov = rho ** np.abs(i[:, None] - i[None, :])   # stationary AR1 covariance
    np.testing.assert_allclose(T @ cov, np.eye(nt), atol=1e-12)


def test_kronecker_logdet_univariate_no_obs():
    wl = W.scaled("pin", 7, 6, 1, 3, 10)
    th = np.array([math.log(1.3), 1.1, math.log(2.5), 0.0])
    p = M.theta_to_params(th, 1)
    Qp = M.prior_precision(wl, th)
    ld = DenseSPD(Qp).logdet()
    ns, nt, a = wl.ns, wl.nt, wl.a
    closed = (ns * nt * math.log(p["tau_u"])
              + ns * ar1_logdet_closed(nt, p["rho"][0])
              + nt * qs_logdet_closed(wl.nx, p["kappa"][0])
              + a * math.log(wl.prior_fixed))
    assert abs(ld - closed) < 1e-11 * abs(closed)
    # marginal variances of the prior: diag(T^-1) = 1, so diag(Q_p^-1) is
    # tau_u^-1 diag(Q_s^-1) repeated over time, then 1/prior_fixed
    d = DenseSPD(Qp).inv_diag()
    want = np.concatenate([np.tile(qs_invdiag_closed(wl.nx, p["kappa"][0]), nt)
                           / p["tau_u"], np.full(a, 1.0 / wl.prior_fixed)])
    np.testing.assert_allclose(d, want, rtol=1e-10)


def test_kronecker_logdet_trivariate_no_obs():
    wl = W.scaled("pin3", 5, 4, 3, 1, 10, seed=3)
    th = wl.theta.copy()
    p = M.theta_to_params(th, 3)
    Qp = M.prior_precision(wl, th)
    ld = DenseSPD(Qp).logdet()
    ns, nt = wl.ns, wl.nt
    closed = sum(ns * ar1_logdet_closed(nt, p["rho"][i])
                 + nt * qs_logdet_closed(wl.nx, p["kappa"][i]) for i in range(3))
    closed += -2.0 * ns * nt * float(np.sum(np.log(p["sigma"])))
    closed += wl.a * math.log(wl.prior_fixed)
    assert abs(ld - closed) < 1e-11 * abs(closed)
    # independent of lambda
    th2 = th.copy()
    th2[9:12] += np.array([0.7, -1.3, 0.4])
    ld2 = DenseSPD(M.prior_precision(wl, th2)).logdet()
    assert abs(ld2 - closed) < 1e-11 * abs(closed)


def test_coregional_eq11_matches_eq6():
    """Eq. 11's printed blocks, and the inverse of the Eq. 6 covariance,
    both against the oracle's mixing weights."""
    s = np.array([0.7, 1.9, 1.2])
    l1, l2, l3 = 0.4, -1.1, 0.8
    Mw = M.mixing_weights(s, np.array([l1, l2, l3]))
    s1, s2, s3 = s ** 2
    # coefficient of Q^i in block (j,k), exactly as printed in Eq. 11
    eq11 = np.zeros((3, 3, 3))
    eq11[0, 0, 0] = 1 / s1; eq11[1, 0, 0] = l1 ** 2 / s2; eq11[2, 0, 0] = l3 ** 2 / s3
    eq11[1, 0, 1] = eq11[1, 1, 0] = -l1 / s2
    eq11[2, 0, 1] = eq11[2, 1, 0] = l2 * l3 / s3
    eq11[2, 0, 2] = eq11[2, 2, 0] = -l3 / s3
    eq11[1, 1, 1] = 1 / s2; eq11[2, 1, 1] = l2 ** 2 / s3
    eq11[2, 1, 2] = eq11[2, 2, 1] = -l2 / s3
    eq11[2, 2, 2] = 1 / s3
    np.testing.assert_allclose(Mw, eq11, rtol=1e-13, atol=1e-15)
    # Eq. 6: Sigma = Lambda blockdiag(Sigma_i) Lambda^T with Eq. 5's Lambda
    rng = np.random.default_rng(0)
    n = 4
    Qi = []
    for _ in range(3):
        B = rng.standard_normal((n, n))
        Qi.append(B @ B.T + n * np.eye(n))
    Lam = np.array([[s[0], 0, 0], [l1 * s[0], s[1], 0],
                    [(l3 + l1 * l2) * s[0], l2 * s[1], s[2]]])
    Sig = np.kron(Lam, np.eye(n)) @ sp.block_diag(
        [np.linalg.inv(q) for q in Qi]).toarray() @ np.kron(Lam, np.eye(n)).T
    Qjoint = np.block([[sum(Mw[i, j, k] * Qi[i] for i in range(3))
                        for k in range(3)] for j in range(3)])
    np.testing.assert_allclose(Qjoint @ Sig, np.eye(3 * n), atol=1e-10)


def test_table2_dimensions():
    with open(os.path.join(GOLDEN, "table2_dims.json")) as f:
        rows = json.load(f)["rows"]
    for r in rows:
        perm = M.bta_permutation(r["nv"], 3, 2, r["nr"])  # structure only
        assert perm.shape[0] == r["nv"] * (3 * 2 + r["nr"])
        b, a = r["nv"] * r["ns"], r["nv"] * r["nr"]
        assert r["nt"] * b + a == r["N"], r["name"]


@pytest.mark.parametrize("nv", [1, 3])
def test_marginal_likelihood_identity(nv):
    """For Gaussian data, f_obj - log p(theta) = log N(y; 0, A Q_p^-1 A^T + D^-1),
    a dense m x m density that never forms Q_c (Eq. 7, 8)."""
    if nv == 1:
        wl = W.scaled("ml1", 5, 4, 1, 2, 60)
    else:
        wl = W.scaled("ml3", 4, 3, 3, 1, 20, seed=5)
    th = wl.theta + 0.1
    parts = F.fobj_parts(wl, th)
    Qp = M.prior_precision(wl, th).toarray()
    A = M.design_matrix(wl).toarray()
    d = M.noise_precision(wl, th)
    y = M.observations(wl)
    S = A @ np.linalg.inv(Qp) @ A.T + np.diag(1.0 / d)
    sign, ldS = np.linalg.slogdet(S)
    assert sign > 0
    m = y.shape[0]
    ll = -0.5 * m * math.log(2 * math.pi) - 0.5 * ldS - 0.5 * y @ np.linalg.solve(S, y)
    got = parts["f"] - parts["log_prior"]
    assert abs(got - ll) < 1e-9 * max(1.0, abs(ll))


def test_x_invariance_and_residual():
    wl = W.config0()
    p = F.fobj_parts(wl, wl.theta, return_factors=True)
    for x in (np.zeros(wl.N), np.random.default_rng(1).standard_normal(wl.N)):
        q = F.fobj_parts(wl, wl.theta, x=x)
        assert abs(q["f"] - p["f"]) < 1e-10 * (abs(p["logdet_p"]) + abs(p["logdet_c"]))
    res = p["Qc"] @ p["mu"] - p["r"]
    assert np.linalg.norm(res) <= 1e-13 * np.linalg.norm(p["r"]) * 1e3


def test_eigen_logdet_and_inverse_small():
    wl = W.scaled("eig", 4, 3, 1, 2, 24)
    Qc = M.conditional_precision(wl, wl.theta).toarray()
    ev = np.linalg.eigvalsh(Qc)
    F1 = DenseSPD(Qc)
    assert abs(F1.logdet() - np.sum(np.log(ev))) < 1e-11 * abs(np.sum(np.log(ev)))
    np.testing.assert_allclose(F1.inv_diag(), np.diag(np.linalg.inv(Qc)), rtol=1e-11)


@pytest.mark.parametrize("nv", [1, 3])
def test_banded_route_equals_dense_route(nv):
    wl = W.scaled("bd", 6, 5, nv, 2, 50, seed=2)
    Qc = M.conditional_precision(wl, wl.theta)
    Fd = DenseSPD(Qc)
    Fb = BandedSPD(Qc, wl.a)
    assert abs(Fd.logdet() - Fb.logdet()) < 1e-12 * abs(Fd.logdet())
    r = np.random.default_rng(0).standard_normal(wl.N)
    np.testing.assert_allclose(Fb.solve(r), Fd.solve(r), rtol=1e-10, atol=1e-12)
    idx = np.array([0, 7, wl.N // 2, wl.N - 1, wl.N - wl.a])
    np.testing.assert_allclose(Fb.inv_diag(idx), Fd.inv_diag(idx), rtol=1e-11)


def test_single_block_reduces_to_lapack():
    """nt = 1: the whole latent field is one block; log|Q| is LAPACK's."""
    wl = W.scaled("one", 6, 1, 1, 2, 20)
    Qc = M.conditional_precision(wl, wl.theta).toarray()
    import scipy.linalg as sla
    L = sla.cholesky(Qc, lower=True)
    assert abs(DenseSPD(Qc).logdet() - 2 * np.sum(np.log(np.diag(L)))) < 1e-12 * 1e3


@pytest.mark.parametrize("nv", [1, 3])
def test_bta_order_gives_bta_pattern(nv):
    """After the permutation of Section IV-B, Q_c is block tridiagonal with an
    arrowhead and Q_p is block tridiagonal (observations stay inside the
    spatial pattern; fixed effects only couple through the arrow)."""
    wl = W.scaled("pat", 5, 4, nv, 2, 30, seed=1)
    perm = M.bta_permutation(nv, wl.ns, wl.nt, wl.nr)
    assert np.array_equal(np.sort(perm), np.arange(wl.N))
    Qp = M.prior_precision(wl, wl.theta)
    Qc = M.conditional_precision(wl, wl.theta, Qp=Qp)
    b, nt = wl.b, wl.nt
    for Q, arrow in ((Qp, False), (Qc, True)):
        Qb = Q[perm][:, perm].tocoo()
        bi = np.minimum(Qb.row // b, nt)
        bj = np.minimum(Qb.col // b, nt)
        inner = (bi < nt) & (bj < nt)
        assert np.all(np.abs(bi[inner] - bj[inner]) <= 1)
        cross = (bi == nt) ^ (bj == nt)
        if not arrow:
            assert not np.any(cross & (Qb.data != 0))
        else:
            assert np.any(cross)
    # observations fall inside the 13-point spatial pattern of Q_s
    A = M.design_matrix(wl)
    G2 = (M.spatial_precision(wl.nx, 1.0) != 0).astype(int)
    AtA = (A.T @ A).tocoo()
    nst = wl.ns * wl.nt
    sel = (AtA.row < nst) & (AtA.col < nst)
    r, c = AtA.row[sel], AtA.col[sel]
    assert np.all(r // wl.ns == c // wl.ns)  # same time step
    assert np.all(np.asarray(G2[r % wl.ns, c % wl.ns]).ravel() == 1)


def test_generator_is_deterministic():
    a = W.config0()
    b = W.config0()
    for ra, rb in zip(a.responses, b.responses):
        for f in ("t", "nodes", "w", "X", "y"):
            assert np.array_equal(getattr(ra, f), getattr(rb, f))
    r = a.responses[0]
    np.testing.assert_allclose(r.w.sum(axis=1), 1.0, atol=1e-15)
    assert np.bincount(r.t).tolist() == [40] * 10


@pytest.mark.parametrize("model", ["separable", "diffusion"])
@pytest.mark.parametrize("nv", [1, 3])
def test_sub_diagonal_blocks_are_symmetric(nv, model):
    """Q(t+1, t) = Q(t, t+1) for every pair of neighbouring time steps, in
    Q_p and Q_c: the coupling blocks are weighted sums of symmetric spatial
    FEM matrices with weights symmetric in the response pair (Eq. 11), and
    observations couple only one time step.  Eliminating the second half of
    the time domain backward uses the assembled B_t as Q(t, t+1)."""
    wl = W.scaled("sym", 5, 4, nv, 2, 40, seed=3, model=model)
    th = wl.theta + 0.1 * np.cos(np.arange(wl.dim_theta))
    perm = M.bta_permutation(nv, wl.ns, wl.nt, wl.nr)
    b = wl.b
    for Q in (M.prior_precision(wl, th), M.conditional_precision(wl, th)):
        Qb = Q[perm][:, perm].toarray()
        for t in range(wl.nt - 1):
            B = Qb[(t + 1) * b:(t + 2) * b, t * b:(t + 1) * b]
            assert np.abs(B).max() > 0
            np.testing.assert_allclose(B, B.T, rtol=0, atol=1e-13 * np.abs(B).max())
