"""Pins of the oracle's optimiser pieces (Eq. 9, 10) and of its FP64
surrogate network, against closed forms, textbook special cases and an
analytic gradient of the Gaussian marginal likelihood."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import bfgs as OB
from oracle import fobj as OF
from oracle import hessian as OH
from oracle import mlp as OL
from oracle import model as OM


def test_central_difference_closed_form():
    """For f = sum x^3 the central difference is 3x^2 + h^2 exactly."""
    x = np.array([0.3, -1.2, 2.0])
    h = 1e-2
    g = OB.central_gradient(lambda v: float(np.sum(v ** 3)), x, h)
    np.testing.assert_allclose(g, 3 * x ** 2 + h ** 2, rtol=1e-12)
    pts = OB.fd_stencil(x, h)
    assert pts.shape == (2 * 3 + 1, 3)   # 2*dim + 1 evaluations


def test_bfgs_quadratic_reaches_solution():
    rng = np.random.default_rng(0)
    B = rng.standard_normal((6, 6))
    A = B @ B.T + 6 * np.eye(6)
    b = rng.standard_normal(6)
    fg = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    x, f, hist = OB.bfgs_minimize(fg, np.zeros(6), max_iter=200, ftol=0, gtol=1e-10)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-7, atol=1e-9)


def test_bfgs_rosenbrock_with_fd_gradient():
    f = lambda v: (1 - v[0]) ** 2 + 100 * (v[1] - v[0] ** 2) ** 2
    fg = lambda v: (f(v), OB.central_gradient(f, v, 1e-6))
    x, fx, _ = OB.bfgs_minimize(fg, np.array([-1.2, 1.0]), max_iter=500, ftol=0,
                                gtol=1e-6)
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-4)


def _analytic_grad_univariate(wl, theta):
    """d f_obj / d theta from f_obj = log p(theta) + log N(y; 0, S),
    S = A Q_p^-1 A^T + D^-1, written from dS/dtheta_k (dense, tiny)."""
    lk, phi, ltu, lty = theta
    kap, rho, tau_u, tau_y = math.exp(lk), math.tanh(phi / 2), math.exp(ltu), math.exp(lty)
    nx, nt, a = wl.nx, wl.nt, wl.a
    C = np.eye(nx * nx)
    G = OM.stiffness_G(nx).toarray()
    Qs = kap ** 4 * C + 2 * kap ** 2 * G + G @ G
    dQs = 4 * kap ** 4 * C + 4 * kap ** 2 * G          # d/d log kappa
    Mr = np.diag(np.r_[1.0, np.full(nt - 2, 1 + rho ** 2), 1.0]) \
        - rho * (np.eye(nt, k=1) + np.eye(nt, k=-1))
    dMr = np.diag(np.r_[0.0, np.full(nt - 2, 2 * rho), 0.0]) \
        - (np.eye(nt, k=1) + np.eye(nt, k=-1))
    T = Mr / (1 - rho ** 2)
    dT = 2 * rho / (1 - rho ** 2) ** 2 * Mr + dMr / (1 - rho ** 2)
    drho = 0.5 * (1 - rho ** 2)
    nst = nx * nx * nt
    def border(Z):
        out = np.zeros((nst + a, nst + a))
        out[:nst, :nst] = Z
        return out
    Qp = border(tau_u * np.kron(T, Qs))
    Qp[nst:, nst:] = wl.prior_fixed * np.eye(a)
    dQ = [border(tau_u * np.kron(T, dQs)), border(tau_u * drho * np.kron(dT, Qs)),
          border(tau_u * np.kron(T, Qs))]
    A = OM.design_matrix(wl).toarray()
    y = OM.observations(wl)
    m = y.shape[0]
    Qi = np.linalg.inv(Qp)
    S = A @ Qi @ A.T + np.eye(m) / tau_y
    Si = np.linalg.inv(S)
    alpha = Si @ y
    g = np.zeros(4)
    for k, dq in enumerate(dQ):
        dS = -A @ Qi @ dq @ Qi @ A.T
        g[k] = -0.5 * np.trace(Si @ dS) + 0.5 * alpha @ dS @ alpha
    dS = -np.eye(m) / tau_y
    g[3] = -0.5 * np.trace(Si @ dS) + 0.5 * alpha @ dS @ alpha
    g -= (theta - wl.theta_prior_mean) / wl.theta_prior_sd ** 2
    return g


def test_fd_gradient_of_fobj_matches_analytic():
    wl = W.scaled("grad", 4, 3, 1, 2, 30, seed=3)
    theta = wl.theta + np.array([0.1, -0.2, 0.15, -0.05])
    g_fd = OB.central_gradient(lambda t: OF.fobj(wl, t), theta, 1e-3)
    g_an = _analytic_grad_univariate(wl, theta)
    np.testing.assert_allclose(g_fd, g_an, rtol=1e-4, atol=1e-4)


# ---- Hessian at the mode (second-order central differences) ---------------------

def test_hessian_stencil_exact_on_quadratics():
    """Second differences are exact for quadratics: H = A; 2 d^2 + 1 points."""
    rng = np.random.default_rng(5)
    B = rng.standard_normal((5, 5))
    A = B + B.T
    b = rng.standard_normal(5)
    f = lambda x: 0.5 * x @ A @ x + b @ x + 3.0
    x0 = rng.standard_normal(5)
    H = OH.hessian(f, x0, 1e-3)
    np.testing.assert_allclose(H, A, atol=1e-7)
    assert OH.hessian_stencil(x0, 1e-3).shape == (2 * 25 + 1, 5)


def test_hessian_stencil_closed_form_separable():
    """f = sum_i exp(c_i x_i) + x_0 x_1^3: the diagonal second difference of
    exp(c x) is exp(c x) (2 cosh(c h) - 2) / h^2 exactly, the mixed one of
    x_0 x_1^3 is 3 x_1^2 + h^2 exactly."""
    c = np.array([0.5, -1.0, 2.0])
    x = np.array([0.3, -0.4, 0.1])
    h = 1e-2
    f = lambda v: float(np.sum(np.exp(c * v)) + v[0] * v[1] ** 3)
    H = OH.hessian(f, x, h)
    diag = np.exp(c * x) * (2.0 * np.cosh(c * h) - 2.0) / h ** 2
    diag[1] += 6.0 * x[0] * x[1]
    np.testing.assert_allclose(np.diag(H), diag, rtol=1e-8)
    np.testing.assert_allclose(H[0, 1], 3 * x[1] ** 2 + h ** 2, rtol=1e-8)
    assert abs(H[0, 2]) < 1e-8 and abs(H[1, 2]) < 1e-8


def test_gaussian_marginal_sd_of_a_gaussian():
    """For a Gaussian log density the approximation is exact."""
    S = np.array([[2.0, 0.3], [0.3, 0.5]])
    P = np.linalg.inv(S)
    logp = lambda x: -0.5 * x @ P @ x
    H = OH.hessian(logp, np.zeros(2), 1e-3)
    np.testing.assert_allclose(OH.gaussian_marginal_sd(H), np.sqrt(np.diag(S)), rtol=1e-6)


def test_fd_hessian_of_fobj_matches_difference_of_analytic_gradient():
    """The second differences of the oracle's f_obj against central
    differences of the analytic gradient of the dense marginal likelihood (a
    different route to the same matrix; both O(h^2))."""
    wl = W.scaled("hess", 4, 3, 1, 2, 30, seed=3)
    theta = wl.theta + np.array([0.1, -0.2, 0.15, -0.05])
    h = 1e-3
    H_fd = OH.hessian(lambda t: OF.fobj(wl, t), theta, h)
    J = np.empty((4, 4))
    for j in range(4):
        e = np.zeros(4)
        e[j] = h
        J[:, j] = (_analytic_grad_univariate(wl, theta + e)
                   - _analytic_grad_univariate(wl, theta - e)) / (2 * h)
    scale = np.max(np.abs(J))
    np.testing.assert_allclose(H_fd, 0.5 * (J + J.T), atol=1e-6 * scale)


# ---- surrogate network -----------------------------------------------------------

def _net(seed=0, sizes=(4, 8, 8, 1)):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((o, i)) / math.sqrt(i), 0.1 * rng.standard_normal(o))
            for i, o in zip(sizes[:-1], sizes[1:])]


def test_silu_gradient():
    z = np.linspace(-4, 4, 17)
    h = 1e-6
    fd = (OL.silu(z + h) - OL.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(OL.silu_grad(z), fd, rtol=1e-8, atol=1e-10)


def test_backward_matches_finite_differences():
    params = _net()
    rng = np.random.default_rng(1)
    X = rng.standard_normal((5, 4))
    y = rng.standard_normal(5)
    loss, grads = OL.mse_loss(params, X, y)
    h = 1e-6
    for k in range(len(params)):
        W, b = params[k]
        for (i, j) in [(0, 0), (W.shape[0] - 1, W.shape[1] - 1), (1 % W.shape[0], 2 % W.shape[1])]:
            Wp, Wm = W.copy(), W.copy()
            Wp[i, j] += h
            Wm[i, j] -= h
            pp = list(params); pp[k] = (Wp, b)
            pm = list(params); pm[k] = (Wm, b)
            fd = (OL.mse_loss(pp, X, y)[0] - OL.mse_loss(pm, X, y)[0]) / (2 * h)
            assert abs(grads[k][0][i, j] - fd) <= 1e-6 * max(1.0, abs(fd))
    # input gradient
    yhat, dX = OL.input_gradient(params, X)
    for j in range(4):
        Xp, Xm = X.copy(), X.copy()
        Xp[:, j] += h
        Xm[:, j] -= h
        fd = (OL.forward(params, Xp)[0] - OL.forward(params, Xm)[0]) / (2 * h)
        np.testing.assert_allclose(dX[:, j], fd, rtol=1e-6, atol=1e-8)


def test_bf16_rounding_against_torch():
    torch = pytest.importorskip("torch")
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.75e-3, 3.1415926, 65504.0,
                     1e-30, -7.77e20], dtype=np.float32)
    want = torch.tensor(vals).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(OL.bf16_round(vals), want)
    assert OL.bf16_round(np.float32(1 + 2 ** -8)) == 1.0        # tie to even
    assert OL.bf16_round(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6


def test_adam_first_step_closed_form():
    """With zero moments, the bias-corrected first step is -lr g/(|g| + eps)."""
    params = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    grads = [(np.array([[0.3, -4.0]]), np.array([1e-3]))]
    state = {}
    OL.adam(params, grads, state, lr=0.01, eps=1e-8)
    W, b = params[0]
    np.testing.assert_allclose(W, [[1.0 - 0.01 * 0.3 / (0.3 + 1e-8),
                                    -2.0 + 0.01 * 4.0 / (4.0 + 1e-8)]], rtol=1e-14)
    np.testing.assert_allclose(b, [0.5 - 0.01 * 1e-3 / (1e-3 + 1e-8)], rtol=1e-14)


# ---- eigenvector reparametrisation of the hyperparameter marginals ----------------

def _random_negdef(d, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    lam = rng.uniform(0.5, 4.0, d)
    return -(Q * lam) @ Q.T, Q, lam


def test_skew_correction_of_a_quadratic_is_gaussian():
    """f quadratic: every axis drops by delta^2/2, so sigma^+- = 1, the points
    lie at Mahalanobis distance delta under -H, and the asymmetric standard
    deviations are the Gaussian marginal ones on both sides."""
    d = 5
    H, _, _ = _random_negdef(d, 3)
    x0 = np.linspace(-1.0, 1.0, d)
    f = lambda t: 7.0 + 0.5 * (t - x0) @ H @ (t - x0)
    A = OH.eigen_axes(H)
    for delta in (1.0, 0.5):
        pts = OH.skew_points(x0, A, delta)
        for p in pts:
            assert abs((p - x0) @ (-H) @ (p - x0) - delta ** 2) < 1e-12
        sp, sm = OH.skew_scales(f(x0), [f(p) for p in pts], delta)
        np.testing.assert_allclose(sp, 1.0, rtol=1e-12)
        np.testing.assert_allclose(sm, 1.0, rtol=1e-12)
        up, dn = OH.asymmetric_sd(A, sp, sm)
        want = np.sqrt(np.diag(np.linalg.inv(-H)))
        np.testing.assert_allclose(up, want, rtol=1e-12)
        np.testing.assert_allclose(dn, want, rtol=1e-12)


def test_skew_correction_recovers_split_normal_scales():
    """f the log density of independent split normals along the axes of a
    known -H (scale s+ on the positive side, s- on the negative side): the
    correction returns exactly those scales, axis by axis (eigen_axes may
    order and orient the axes differently: matched by direction)."""
    d = 4
    H, Q, lam = _random_negdef(d, 8)
    rng = np.random.default_rng(9)
    s_plus = rng.uniform(0.5, 2.0, d)
    s_minus = rng.uniform(0.5, 2.0, d)
    x0 = rng.standard_normal(d)

    def f(t):
        z = np.sqrt(lam) * (Q.T @ (t - x0))   # coordinates with -H = Q lam Q^T
        s = np.where(z >= 0.0, s_plus, s_minus)
        return -0.5 * np.sum((z / s) ** 2)

    A = OH.eigen_axes(H)
    pts = OH.skew_points(x0, A, 1.0)
    sp, sm = OH.skew_scales(f(x0), [f(p) for p in pts], 1.0)
    V = A * np.sqrt(np.linalg.eigvalsh(-H))[None, :]     # unit eigenvectors
    for k in range(d):
        dots = Q.T @ V[:, k]
        j = int(np.argmax(np.abs(dots)))
        assert abs(abs(dots[j]) - 1.0) < 1e-10
        want_p, want_m = (s_plus[j], s_minus[j]) if dots[j] > 0 else (s_minus[j], s_plus[j])
        assert abs(sp[k] - want_p) < 1e-10 and abs(sm[k] - want_m) < 1e-10


def test_skew_correction_in_one_dimension_is_the_split_normal():
    """d = 1: theta = theta* + a z with z split normal; the upper and lower
    standard deviations of theta are a s+ and a s-."""
    a, s_plus, s_minus, x0 = 0.7, 1.6, 0.6, 0.3
    H = np.array([[-1.0 / a ** 2]])
    f = lambda t: -0.5 * (((t[0] - x0) / a) / (s_plus if t[0] >= x0 else s_minus)) ** 2
    A = OH.eigen_axes(H)
    pts = OH.skew_points(np.array([x0]), A, 1.0)
    sp, sm = OH.skew_scales(f(np.array([x0])), [f(p) for p in pts], 1.0)
    up, dn = OH.asymmetric_sd(A, sp, sm)
    assert abs(up[0] - a * s_plus) < 1e-12 and abs(dn[0] - a * s_minus) < 1e-12
    with pytest.raises(ValueError):
        OH.skew_scales(0.0, [0.5, -1.0], 1.0)     # f rises: not a mode


def test_gpu_hessian_driver_host_logic_matches_oracle():
    """The Hessian driver's host-side steps (stencil order, second
    differences, reparametrisation axes, asymmetric standard deviations)
    against the oracle's independent code, on synthetic values."""
    from paper_2507_06938_amd import hessian as GH
    rng = np.random.default_rng(17)
    d, h = 4, 1e-3
    x = rng.standard_normal(d)
    np.testing.assert_array_equal(GH.stencil_points(x, h), OH.hessian_stencil(x, h))
    vals = rng.standard_normal(2 * d * d + 1)
    np.testing.assert_allclose(GH.second_differences(vals, d, h),
                               OH.hessian_from_values(vals, d, h), rtol=1e-12, atol=1e-6)
    H = -(lambda B: B @ B.T + d * np.eye(d))(rng.standard_normal((d, d)))
    np.testing.assert_allclose(GH.reparam_axes(H), OH.eigen_axes(H), rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(GH.marginal_sd(H), OH.gaussian_marginal_sd(H), rtol=1e-12)
    A = OH.eigen_axes(H)
    sp, sm = rng.uniform(0.5, 2.0, d), rng.uniform(0.5, 2.0, d)
    for got, want in zip(GH.skew_sd(A, sp, sm), OH.asymmetric_sd(A, sp, sm)):
        np.testing.assert_allclose(got, want, rtol=1e-12)
    with pytest.raises(ValueError):
        GH.reparam_axes(-H)


class _AnalyticEvaluator:
    """Stands in for the batched GPU evaluator of the mode-search driver:
    the same call interface (rows of theta in, values of F out, `ntrial`
    points per line-search pass, a running count), values from a smooth
    analytic function."""

    def __init__(self, F, ntrial=4):
        self.F = F
        self.ntrial = ntrial
        self.count = 0

    def __call__(self, thetas):
        thetas = np.atleast_2d(np.asarray(thetas, np.float64))
        self.count += thetas.shape[0]
        return np.array([self.F(t) for t in thetas])


def _smooth_convex(d, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((d, d))
    A = B @ B.T / d + 0.5 * np.eye(d)
    b = rng.standard_normal(d)
    return lambda x: float(0.5 * x @ A @ x - b @ x + 0.3 * np.sum(np.log(np.cosh(2.0 * x))))


@pytest.mark.parametrize("d,seed,x0", [(4, 31, 3.0), (6, 32, -2.5)])
def test_fd_bfgs_driver_host_logic_matches_oracle(d, seed, x0):
    """The mode-search driver's host-side steps (stencil, Eq. 10 gradient,
    capped quasi-Newton direction, Armijo ladder evaluated a pass at a time,
    scaled first inverse Hessian, stopping rule) follow the oracle's BFGS
    iterate for iterate: on the same function both visit the same points."""
    from paper_2507_06938_amd import optimize as GO
    F = _smooth_convex(d, seed)
    h = 1e-3
    theta0 = np.full(d, x0) + 0.1 * np.arange(d)
    np.testing.assert_array_equal(GO.fd_points(theta0, h), OB.fd_stencil(theta0, h))
    vals = np.array([F(p) for p in OB.fd_stencil(theta0, h)])
    ev = _AnalyticEvaluator(F)
    F0, g0 = GO.fd_gradient(ev, theta0, h)
    assert F0 == vals[0] and ev.count == 2 * d + 1
    np.testing.assert_array_equal(g0, OB.central_gradient_from_values(vals, h))

    ev = _AnalyticEvaluator(F)
    tr = GO.fd_bfgs(ev, theta0, h=h, ftol=1e-12, gtol=1e-7, max_iter=60)
    fg = lambda t: (F(t), OB.central_gradient(F, t, h))
    x_ref, f_ref, hist = OB.bfgs_minimize(fg, theta0, max_iter=60, ftol=1e-12, gtol=1e-7)
    assert len(tr.theta) == len(hist) > 3
    for k, (x, rec) in enumerate(zip(tr.theta, hist)):
        np.testing.assert_allclose(x, rec["x"], rtol=1e-13, atol=1e-13, err_msg=str(k))
        assert abs(tr.f[k] - rec["f"]) <= 1e-13 * max(1.0, abs(rec["f"])), k
    # the start is several unit steps from the mode: the cap was active
    assert np.linalg.norm(tr.theta[1] - tr.theta[0]) == pytest.approx(1.0, abs=1e-12)
