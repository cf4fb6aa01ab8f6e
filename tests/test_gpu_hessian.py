"""Hessian of f at the mode (second-order central differences over batched
GPU f_obj values) against the oracle's second differences of its FP64 f_obj,
on a tiny univariate model at the oracle's optimum.

Tolerance: every entry is a sum of four values over 4 h^2 (or three over
h^2), so a value error delta gives at most delta / h^2 in H; the GPU and
oracle f_obj agree to ~1e-13 relative here, and the bound allows 2e-12:
|H_gpu - H_oracle| <= 2e-12 |f| / h^2.  Both Hessians must be negative
definite at the mode, and their Gaussian marginal standard deviations agree.
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


def test_hessian_at_mode_matches_oracle(mode):
    import torch
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
