"""Pins of the oracle's non-separable (diffusion-based) space-time model.

The model is a sum of Kronecker products of temporal and spatial FEM matrices
(Section IV-B, multivariate model formulation).  The oracle assembles it as sparse
matrix products; these checks reach the same numbers by other routes:

  * the temporal FEM matrices against the integrals they discretise, on
    piecewise-linear paths;
  * the quadratic form on a separable vector (a time path times a spatial
    eigenvector) against the continuous operator (gamma_t d/dt + L) with
    noise precision L, integrated exactly where the FEM is exact and by the
    trapezoid rule where the mass matrix is lumped;
  * the log-determinant and the marginal variances from the closed-form
    spectrum of the grid Laplacian (DCT eigenpairs), one small temporal
    matrix per spatial mode obtained by polarising that quadratic form;
  * the gamma_t -> 0 limit (independent time slices of a Matern field with
    spectrum (gamma_s^2 + lambda)^3);
  * the Gaussian marginal likelihood written without Q_c, and the block
    tridiagonal pattern after the BTA permutation.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import model as M
from oracle import fobj as F
from oracle.linalg import DenseSPD, BandedSPD


def dct_eigs(nx):
    k = np.arange(nx)
    return 2.0 - 2.0 * np.cos(np.pi * k / nx)


def dct_basis(nx):
    i = np.arange(nx)[:, None]
    k = np.arange(nx)[None, :]
    V = np.cos(np.pi * k * (i + 0.5) / nx) * math.sqrt(2.0 / nx)
    V[:, 0] = 1.0 / math.sqrt(nx)
    return V


def continuous_qform(a, e, gamma_t):
    """e * [ int (gamma_t a' + e a)^2 dt + boundary ] for a piecewise-linear
    path a on unit-spaced nodes, with the integral of a a' taken exactly and
    the stationary start adding gamma_t e a(0)^2:
        gamma_t^2 int a'^2 + gamma_t e (a(0)^2 + a(T)^2) + e^2 int a^2,
    where int a'^2 is exact for piecewise-linear a and int a^2 is the
    trapezoid rule (lumped mass)."""
    a = np.asarray(a, np.float64)
    da = np.diff(a)
    int_da2 = float(np.sum(da * da))
    trap = float(np.sum(0.5 * (a[:-1] ** 2 + a[1:] ** 2)))
    return e * (gamma_t ** 2 * int_da2 + gamma_t * e * (a[0] ** 2 + a[-1] ** 2)
                + e * e * trap)


def mode_matrix(nt, e, gamma_t):
    """nt x nt matrix of the quadratic form above, by polarisation."""
    I = np.eye(nt)
    q = [continuous_qform(I[i], e, gamma_t) for i in range(nt)]
    A = np.diag(q)
    for i in range(nt):
        for j in range(i + 1, nt):
            v = 0.5 * (continuous_qform(I[i] + I[j], e, gamma_t) - q[i] - q[j])
            A[i, j] = A[j, i] = v
    return A


def spectral_logdet(nx, nt, gamma_s, gamma_t):
    lam = dct_eigs(nx)
    tot = 0.0
    for lx in lam:
        for ly in lam:
            sign, ld = np.linalg.slogdet(mode_matrix(nt, gamma_s ** 2 + lx + ly,
                                                     gamma_t))
            assert sign > 0
            tot += ld
    return tot


def spectral_invdiag(nx, nt, gamma_s, gamma_t):
    """diag(Q^-1) at index t*ns + s (time outermost, node s = iy*nx + ix)."""
    lam = dct_eigs(nx)
    V = dct_basis(nx)
    ns = nx * nx
    out = np.zeros(nt * ns)
    for kx in range(nx):
        for ky in range(nx):
            Ai = np.diag(np.linalg.inv(mode_matrix(nt, gamma_s ** 2 + lam[kx]
                                                   + lam[ky], gamma_t)))
            v2 = np.outer(V[:, ky] ** 2, V[:, kx] ** 2).ravel()   # (iy, ix)
            out += np.kron(Ai, v2)
    return out


# ---- temporal FEM ------------------------------------------------------------------

@pytest.mark.parametrize("nt", [2, 3, 9])
def test_temporal_fem_integrals(nt):
    M0, M1, M2 = (X.toarray() for X in M.temporal_fem(nt))
    rng = np.random.default_rng(nt)
    for _ in range(5):
        a = rng.standard_normal(nt)
        assert abs(a @ M2 @ a - np.sum(np.diff(a) ** 2)) < 1e-12
        trap = np.sum(0.5 * (a[:-1] ** 2 + a[1:] ** 2))
        assert abs(a @ M0 @ a - trap) < 1e-12
        assert abs(a @ M1 @ a - 0.5 * (a[0] ** 2 + a[-1] ** 2)) < 1e-12
    one = np.ones(nt)
    assert abs(one @ M0 @ one - (nt - 1)) < 1e-12     # length of the interval
    np.testing.assert_allclose(M2 @ one, 0.0, atol=1e-15)
    t = np.arange(nt, dtype=np.float64)
    flux = np.zeros(nt)
    flux[0], flux[-1] = -1.0, 1.0
    np.testing.assert_allclose(M2 @ t, flux, atol=1e-12)
    with pytest.raises(ValueError):
        M.temporal_fem(1)


# ---- the space-time operator ---------------------------------------------------------

@pytest.mark.parametrize("gamma_s,gamma_t", [(1.0, 2.0), (0.5, 0.3), (2.0, 4.0)])
def test_diffusion_quadratic_form_on_separable_vectors(gamma_s, gamma_t):
    nx, nt = 5, 6
    Q = M.diffusion_precision(nx, nt, gamma_s, gamma_t)
    lam = dct_eigs(nx)
    V = dct_basis(nx)
    rng = np.random.default_rng(7)
    for kx, ky in ((0, 0), (1, 0), (2, 3), (4, 4)):
        v = np.outer(V[:, ky], V[:, kx]).ravel()      # node s = iy*nx + ix
        e = gamma_s ** 2 + lam[kx] + lam[ky]
        a = rng.standard_normal(nt)
        x = np.kron(a, v)                              # index t*ns + s
        got = float(x @ (Q @ x))
        want = continuous_qform(a, e, gamma_t)
        assert abs(got - want) < 1e-11 * max(1.0, abs(want)), (kx, ky)


@pytest.mark.parametrize("nx,nt,gamma_s,gamma_t",
                         [(4, 2, 1.0, 2.0), (5, 5, 0.7, 1.3), (6, 4, 1.5, 0.4)])
def test_diffusion_spectral_logdet_and_variances(nx, nt, gamma_s, gamma_t):
    Q = M.diffusion_precision(nx, nt, gamma_s, gamma_t).toarray()
    sign, ld = np.linalg.slogdet(Q)
    assert sign > 0
    closed = spectral_logdet(nx, nt, gamma_s, gamma_t)
    assert abs(ld - closed) < 1e-11 * abs(closed)
    np.testing.assert_allclose(np.diag(np.linalg.inv(Q)),
                               spectral_invdiag(nx, nt, gamma_s, gamma_t),
                               rtol=1e-10)


def test_diffusion_without_time_coupling_is_a_matern_field_per_step():
    """gamma_t = 0 leaves M0 (x) K_3: independent time slices, each with the
    spectrum (gamma_s^2 + lambda)^3 scaled by the lumped time mass."""
    nx, nt, gs = 5, 4, 0.8
    Q = M.diffusion_precision(nx, nt, gs, 0.0).toarray()
    lam = dct_eigs(nx)
    e = (gs ** 2 + lam[:, None] + lam[None, :]).ravel()
    ns = nx * nx
    m0 = np.array([0.5] + [1.0] * (nt - 2) + [0.5])
    closed = ns * float(np.sum(np.log(m0))) + nt * float(np.sum(3 * np.log(e)))
    sign, ld = np.linalg.slogdet(Q)
    assert sign > 0 and abs(ld - closed) < 1e-11 * abs(closed)
    off = Q[:ns, ns:]
    assert np.abs(off).max() == 0.0


def test_diffusion_univariate_prior_logdet():
    wl = W.scaled("dpin", 5, 4, 1, 2, 10, model="diffusion")
    th = np.array([math.log(1.3), math.log(0.6), math.log(2.5), 0.0])
    p = M.theta_to_params(th, 1, "diffusion")
    Qp = M.prior_precision(wl, th)
    F1 = DenseSPD(Qp)
    ns, nt, a = wl.ns, wl.nt, wl.a
    closed = (ns * nt * math.log(p["tau_u"])
              + spectral_logdet(wl.nx, nt, p["gamma_s"][0], p["gamma_t"][0])
              + a * math.log(wl.prior_fixed))
    assert abs(F1.logdet() - closed) < 1e-11 * abs(closed)
    want = np.concatenate([
        spectral_invdiag(wl.nx, nt, p["gamma_s"][0], p["gamma_t"][0]) / p["tau_u"],
        np.full(a, 1.0 / wl.prior_fixed)])
    np.testing.assert_allclose(F1.inv_diag(), want, rtol=1e-10)


def test_diffusion_trivariate_prior_logdet():
    wl = W.scaled("dpin3", 4, 3, 3, 1, 10, seed=3, model="diffusion")
    th = wl.theta.copy()
    p = M.theta_to_params(th, 3, "diffusion")
    ns, nt = wl.ns, wl.nt
    closed = sum(spectral_logdet(wl.nx, nt, p["gamma_s"][i], p["gamma_t"][i])
                 for i in range(3))
    closed += -2.0 * ns * nt * float(np.sum(np.log(p["sigma"])))
    closed += wl.a * math.log(wl.prior_fixed)
    ld = DenseSPD(M.prior_precision(wl, th)).logdet()
    assert abs(ld - closed) < 1e-11 * abs(closed)
    th2 = th.copy()
    th2[9:12] += np.array([0.5, -0.9, 1.1])        # lambda does not enter
    ld2 = DenseSPD(M.prior_precision(wl, th2)).logdet()
    assert abs(ld2 - closed) < 1e-11 * abs(closed)


@pytest.mark.parametrize("nv", [1, 3])
def test_diffusion_marginal_likelihood_identity(nv):
    """f_obj - log p(theta) = log N(y; 0, A Q_p^-1 A^T + D^-1) (Eq. 7, 8)."""
    if nv == 1:
        wl = W.scaled("dml1", 5, 4, 1, 2, 60, model="diffusion")
    else:
        wl = W.scaled("dml3", 4, 3, 3, 1, 20, seed=5, model="diffusion")
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
    assert abs(parts["f"] - parts["log_prior"] - ll) < 1e-9 * max(1.0, abs(ll))


@pytest.mark.parametrize("nv", [1, 3])
def test_diffusion_bta_pattern_and_banded_route(nv):
    """The wider spatial stencil stays inside each time block; time coupling
    stays nearest-neighbour, so the BTA permutation still gives the block
    tridiagonal pattern, and the banded route agrees with the dense one."""
    wl = W.scaled("dpat", 6, 4, nv, 2, 40, seed=1, model="diffusion")
    perm = M.bta_permutation(nv, wl.ns, wl.nt, wl.nr)
    Qc = M.conditional_precision(wl, wl.theta)
    Qb = Qc[perm][:, perm].tocoo()
    b, nt = wl.b, wl.nt
    bi = np.minimum(Qb.row // b, nt)
    bj = np.minimum(Qb.col // b, nt)
    inner = (bi < nt) & (bj < nt)
    assert np.all(np.abs(bi[inner] - bj[inner]) <= 1)
    # spatial reach: L1 distance 3 on the grid (G C^-1 G C^-1 G)
    nst = wl.ns * wl.nt
    Qpc = M.prior_precision(wl, wl.theta).tocoo()
    sel = (Qpc.row < nst) & (Qpc.col < nst) & (Qpc.data != 0)
    sr, sc = Qpc.row[sel] % wl.ns, Qpc.col[sel] % wl.ns
    dist = np.abs(sr % wl.nx - sc % wl.nx) + np.abs(sr // wl.nx - sc // wl.nx)
    assert dist.max() == 3
    Fd = DenseSPD(Qc)
    Fb = BandedSPD(Qc, wl.a)
    assert abs(Fd.logdet() - Fb.logdet()) < 1e-12 * abs(Fd.logdet())
    idx = np.array([0, 5, wl.N // 2, wl.N - 1])
    np.testing.assert_allclose(Fb.inv_diag(idx), Fd.inv_diag(idx), rtol=1e-11)
