"""Hessian of f at the mode (second-order central differences over batched
GPU f_obj values) against the oracle's second differences of its FP64 f_obj,
on a tiny univariate model at the oracle's optimum.

Tolerance: every entry is a sum of four values over 4 h^2 (or three over
h^2), so a value error delta gives at most delta / h^2 in H; the GPU and
oracle f_obj agree to ~1e-13 relative here, and the bound allows 2e-12:
|H_gpu - H_oracle| <= 2e-12 |f| / h^2.  Both Hessians must be negative
definite at the mode, and their Gaussian marginal standard deviations agree.

The eigenvector reparametrisation (split-normal scales along the axes of
-H, from 2 d more values) is compared with the oracle's on the same mode:
the axes follow from the two Hessians, which agree to ~1e-8 relative, so
the scales and asymmetric standard deviations are compared to 1e-5.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bfgs as OB
from oracle import fobj as OF
from oracle import hessian as OH

pytestmark = pytest.mark.gpu
H_STEP = 1e-3


@pytest.fixture(scope="module")
def mode():
    wl = W.scaled("hess_tiny", 5, 4, 1, 2, 60, seed=11)
    F = lambda t: -OF.fobj(wl, t)
    fg = lambda t: (F(t), OB.central_gradient(F, t, 1e-3))
    x, f, _ = OB.bfgs_minimize(fg, wl.theta.copy(), max_iter=300, ftol=1e-13, gtol=1e-6)
    return wl, x


@pytest.fixture(scope="module")
def hess(mode):
    from paper_2507_06938_amd import dalia as D
    from paper_2507_06938_amd import hessian as GH
    wl, xs = mode
    d = wl.dim_theta
    model = D.Model.from_workload(wl)
    ws = D.Workspace([model] * (2 * d + 1))
    H_gpu, f0, vals = GH.fobj_hessian(ws, xs, H_STEP)
    pts = OH.hessian_stencil(xs, H_STEP)
    ref_vals = np.array([OF.fobj(wl, p) for p in pts])
    H_ref = OH.hessian_from_values(ref_vals, d, H_STEP)
    return ws, H_gpu, f0, vals, ref_vals, H_ref


def test_hessian_at_mode_matches_oracle(mode, hess):
    from paper_2507_06938_amd import hessian as GH
    wl, xs = mode
    d = wl.dim_theta
    ws, H_gpu, f0, vals, ref_vals, H_ref = hess
    dv = np.max(np.abs(vals - ref_vals)) / abs(ref_vals[0])
    dh = np.max(np.abs(H_gpu - H_ref))
    print(f"f={f0:.12f}  max rel f diff {dv:.2e}  max |dH| {dh:.2e}  "
          f"points {vals.size}", flush=True)
    assert vals.size == 2 * d * d + 1
    assert dh <= 2e-12 * abs(ref_vals[0]) / H_STEP ** 2
    assert np.linalg.eigvalsh(H_ref).max() < 0
    assert np.linalg.eigvalsh(H_gpu).max() < 0
    np.testing.assert_allclose(GH.marginal_sd(H_gpu), OH.gaussian_marginal_sd(H_ref),
                               rtol=1e-4)


def test_skew_reparametrisation_at_mode_matches_oracle(mode, hess):
    from paper_2507_06938_amd import hessian as GH
    wl, xs = mode
    d = wl.dim_theta
    ws, H_gpu, f0, vals, ref_vals, H_ref = hess
    A, sp, sm, sv = GH.fobj_skew(ws, xs, H_gpu, f0)
    A_ref = OH.eigen_axes(H_ref)
    pts = OH.skew_points(xs, A_ref, 1.0)
    sp_ref, sm_ref = OH.skew_scales(ref_vals[0], [OF.fobj(wl, p) for p in pts], 1.0)
    print("scales +", sp, "oracle", sp_ref, "\nscales -", sm, "oracle", sm_ref, flush=True)
    assert sv.size == 2 * d and sp is not None
    np.testing.assert_allclose(A, A_ref, rtol=1e-5, atol=1e-8 * np.abs(A_ref).max())
    np.testing.assert_allclose(sp, sp_ref, rtol=1e-5)
    np.testing.assert_allclose(sm, sm_ref, rtol=1e-5)
    up, dn = GH.skew_sd(A, sp, sm)
    up_ref, dn_ref = OH.asymmetric_sd(A_ref, sp_ref, sm_ref)
    np.testing.assert_allclose(up, up_ref, rtol=1e-5)
    np.testing.assert_allclose(dn, dn_ref, rtol=1e-5)
    # the posterior is not exactly Gaussian: the scales depart from 1
    assert np.max(np.abs(np.concatenate([sp, sm]) - 1.0)) > 1e-4
