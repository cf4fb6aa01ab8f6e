"""Write the stored expected values of the full-size parity tests.

    python tests/golden/make_golden.py c1 [c2] [c1_diffusion] [c1_poisson] [c2_poisson]
    python tests/golden/make_golden.py opt_tri

Calls only the CPU oracle (``oracle/``) on the seeded workloads of
``workloads/``; nothing here touches the GPU path.  For each configuration it
stores log|Q_p|, log|Q_c|, the parts of f_obj, and the conditional mean and
the marginal variances diag(Q_c^{-1}) at seeded sample positions (BTA order,
plus every fixed effect), computed with the RCM + banded LAPACK route.  For
the Poisson workload the mean is the inner mode and the variances are those
of the Laplace approximation, diag(Q_c(x*)^{-1}); the Newton step count is
stored too.  ``opt_tri`` stores the mode of a small trivariate model
(dim theta = 15, the surrogate's input width) found by the oracle's BFGS on
its own f_obj with central differences (Eq. 9, 10), from a seeded start.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import fobj as OF  # noqa: E402
from oracle import model as OM  # noqa: E402

CONFIGS = {"c1": W.config1, "c2": W.config2,
           "c1_diffusion": lambda: W.config1(model="diffusion"),
           "c1_poisson": lambda: W.config1(likelihood="poisson"),
           "c2_poisson": lambda: W.config2(likelihood="poisson")}


def sample_positions(N, a, k, seed):
    rng = np.random.default_rng(seed)
    idx = rng.choice(N - a, size=k, replace=False)
    return np.sort(np.concatenate([idx, np.arange(N - a, N)])).astype(np.int64)


def make(name):
    wl = CONFIGS[name]()
    t0 = time.time()
    p = OF.fobj_parts(wl, wl.theta, method="banded", return_factors=True)
    t1 = time.time()
    perm = OM.bta_permutation(wl.nv, wl.ns, wl.nt, wl.nr)
    mu_bta = p["mu"][perm]
    mu_idx = sample_positions(wl.N, wl.a, 256, 1)
    var_idx = sample_positions(wl.N, wl.a, 48, 2)
    var = p["Fc"].inv_diag(perm[var_idx])
    t2 = time.time()
    out = dict(
        workload=wl.name, N=int(wl.N), theta=wl.theta.tolist(),
        logdet_p=p["logdet_p"], logdet_c=p["logdet_c"], f=p["f"],
        quad_p=p["quad_p"], quad_obs=p["quad_obs"], log_prior=p["log_prior"],
        log_lik=p["log_lik"],
        mu_index_bta=mu_idx.tolist(), mu=mu_bta[mu_idx].tolist(),
        var_index_bta=var_idx.tolist(), var=var.tolist(),
        oracle="RCM + LAPACK banded Cholesky (dpbtrf) with a Schur border",
        bandwidth_Qc=int(p["Fc"].kd),
        newton_steps=int(p.get("newton_steps", 0)),
        seconds=dict(fobj=t1 - t0, variances=t2 - t1),
    )
    path = os.path.join(HERE, f"{name}_golden.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: f={out['f']:.10f} ld_p={out['logdet_p']:.6f} "
          f"ld_c={out['logdet_c']:.6f} ({t1 - t0:.1f}s + {t2 - t1:.1f}s) -> {path}")


def opt_tri_workload():
    """The small trivariate model of the mode-search test (15 hyperparameters)."""
    return W.scaled("opt_tri", 5, 4, 3, 2, 60, seed=11)


def make_opt_tri():
    from oracle import bfgs as OB
    wl = opt_tri_workload()
    theta0 = W.random_theta_near(wl.theta, 0.25, seed=3)
    F = lambda t: -OF.fobj(wl, t)
    fg = lambda t: (F(t), OB.central_gradient(F, t, 1e-3))
    t0 = time.time()
    x, f, hist = OB.bfgs_minimize(fg, theta0, max_iter=300, ftol=1e-13, gtol=1e-6)
    out = dict(workload=wl.name, dim_theta=int(wl.dim_theta), theta0=theta0.tolist(),
               theta_star=np.asarray(x).tolist(), F_star=float(f), iterations=len(hist) - 1,
               oracle="BFGS on the oracle's f_obj, central differences h = 1e-3",
               seconds=time.time() - t0)
    path = os.path.join(HERE, "opt_tri_optimum.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"opt_tri: F*={out['F_star']:.12f} in {out['iterations']} iterations -> {path}")


if __name__ == "__main__":
    for n in sys.argv[1:] or ["c1"]:
        make_opt_tri() if n == "opt_tri" else make(n)
