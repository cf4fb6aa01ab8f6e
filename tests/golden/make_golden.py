"""Write the stored expected values of the full-size parity tests.

    python tests/golden/make_golden.py c1 [c2] [c1_diffusion] [c1_poisson] [c2_poisson]

Calls only the CPU oracle (``oracle/``) on the seeded workloads of
``workloads/``; nothing here touches the GPU path.  For each configuration it
stores log|Q_p|, log|Q_c|, the parts of f_obj, and the conditional mean and
the marginal variances diag(Q_c^{-1}) at seeded sample positions (BTA order,
plus every fixed effect), computed with the RCM + banded LAPACK route.  For
the Poisson workload the mean is the inner mode and the variances are those
of the Laplace approximation, diag(Q_c(x*)^{-1}); the Newton step count is
stored too.
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


if __name__ == "__main__":
    for n in sys.argv[1:] or ["c1"]:
        make(n)
