"""Hessian of f at the mode and the Gaussian approximation of the
hyperparameter marginals (Sec. III, marginal posteriors of the hyperparameters), on the batched GPU evaluator.

The second-order central differences with step h on the internal theta --
    H_ii = (f(x + h e_i) - 2 f(x) + f(x - h e_i)) / h^2,
    H_ij = (f(x + h e_i + h e_j) - f(x + h e_i - h e_j)
            - f(x - h e_i + h e_j) + f(x - h e_i - h e_j)) / (4 h^2)
-- need 2 d^2 + 1 independent f_obj values; they are evaluated as batched
passes of the library (a workspace of `batch` instances, the last pass
padded).  The Gaussian approximation of the marginals has covariance
(-H)^{-1} at the mode.

Skewed marginals (the eigenvector reparametrisation the paper cites from
Martins et al., 2013): in the coordinates z with theta = theta* + A z,
A = V diag(lambda)^{-1/2} for -H = V diag(lambda) V^T, the Gaussian
approximation is standard; f_obj at z = +-delta e_k (2 d more values, one
batched pass for d <= batch/2) gives each axis a scale per side,
delta / sqrt(2 (f(theta*) - f)), 1 for an exactly Gaussian posterior, and
the upper (lower) standard deviation of theta_j sums A_jk^2 times the
squared scale of the side of axis k that raises (lowers) theta_j.

Host-side logic only; every f_obj value comes from the library's kernels.

    python -m paper_2507_06938_amd.hessian [c1|c2|c1_poisson] [--batch B]

(c1_poisson: the c1 mesh with counts; the batch workspace warm-starts each
instance's inner Newton search from its previous mode.)

prints one JSON document: the Hessian at the workload's generator theta,
its eigenvalues, the evaluations and their rate.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np


def stencil_points(theta: np.ndarray, h: float) -> np.ndarray:
    """x, then x +- h e_i, then for each i < j the corners in the order
    (+,+), (+,-), (-,+), (-,-)."""
    x = np.asarray(theta, np.float64)
    d = x.size
    rows = [x]
    for i in range(d):
        e = np.zeros(d)
        e[i] = h
        rows += [x + e, x - e]
    for i in range(d):
        ei = np.zeros(d)
        ei[i] = h
        for j in range(i + 1, d):
            ej = np.zeros(d)
            ej[j] = h
            rows += [x + ei + ej, x + ei - ej, x - ei + ej, x - ei - ej]
    return np.array(rows)


def second_differences(f: np.ndarray, d: int, h: float) -> np.ndarray:
    """H from the values at stencil_points (same order)."""
    H = np.zeros((d, d))
    c = f[0]
    for i in range(d):
        H[i, i] = (f[1 + 2 * i] - 2.0 * c + f[2 + 2 * i]) / h ** 2
    pos = 1 + 2 * d
    for i in range(d):
        for j in range(i + 1, d):
            q = f[pos:pos + 4]
            H[i, j] = ((q[0] - q[1]) - (q[2] - q[3])) / (4.0 * h ** 2)
            H[j, i] = H[i, j]
            pos += 4
    return H


def batched_values(ws, pts: np.ndarray) -> np.ndarray:
    """f_obj at the rows of pts in passes of the workspace `ws` (all
    instances of one model; the last pass padded with copies of its first
    point)."""
    import torch
    B = ws.B
    vals = np.empty(pts.shape[0])
    for k0 in range(0, pts.shape[0], B):
        chunk = pts[k0:k0 + B]
        n = chunk.shape[0]
        if n < B:
            chunk = np.concatenate([chunk, np.repeat(chunk[:1], B - n, axis=0)])
        f, _, info = ws.fobj(chunk)
        vals[k0:k0 + n] = f.cpu().numpy()[:n]
    torch.cuda.synchronize()
    return vals


def fobj_hessian(ws, theta: np.ndarray, h: float = 1e-3):
    """(H, f(theta), values) of f_obj at theta from batched passes of the
    workspace `ws` (all instances of one model); values: f_obj at the
    stencil points."""
    pts = stencil_points(theta, h)
    vals = batched_values(ws, pts)
    return second_differences(vals, pts.shape[1], h), vals[0], vals


def reparam_axes(H: np.ndarray) -> np.ndarray:
    """Columns V_k / sqrt(lambda_k) for -H = V diag(lambda) V^T, eigenvalues
    ascending, each column oriented so that its largest-magnitude entry is
    positive.  Raises ValueError unless H is negative definite."""
    lam, V = np.linalg.eigh(-H)
    if not np.all(lam > 0.0):
        raise ValueError("Hessian not negative definite")
    cols = np.arange(V.shape[1])
    sign = np.sign(V[np.abs(V).argmax(axis=0), cols])
    return V * (sign / np.sqrt(lam))[None, :]


def fobj_skew(ws, theta: np.ndarray, H: np.ndarray, f0: float, delta: float = 1.0):
    """(A, scale_plus, scale_minus, values): f_obj at theta +- delta A e_k
    (rows alternate + and - per axis) and the split-normal scale of each
    axis per side; the scales are None when f does not drop along every
    axis (theta is then not a mode)."""
    A = reparam_axes(H)
    d = A.shape[1]
    pts = np.empty((2 * d, d))
    pts[0::2] = theta[None, :] + delta * A.T
    pts[1::2] = theta[None, :] - delta * A.T
    vals = batched_values(ws, pts)
    drop = f0 - vals
    if not np.all(drop > 0.0):
        return A, None, None, vals
    scale = delta / np.sqrt(2.0 * drop)
    return A, scale[0::2], scale[1::2], vals


def skew_sd(A: np.ndarray, scale_plus: np.ndarray, scale_minus: np.ndarray):
    """(upper, lower) standard deviations of every theta_j."""
    sq_p, sq_m = scale_plus ** 2, scale_minus ** 2
    raise_side = np.where(A >= 0.0, sq_p[None, :], sq_m[None, :])
    lower_side = np.where(A >= 0.0, sq_m[None, :], sq_p[None, :])
    A2 = A * A
    return np.sqrt((A2 * raise_side).sum(axis=1)), np.sqrt((A2 * lower_side).sum(axis=1))


def marginal_sd(H: np.ndarray) -> np.ndarray:
    """Marginal standard deviations of the Gaussian with covariance (-H)^{-1}."""
    return np.sqrt(np.diag(np.linalg.inv(-H)))


def main(argv=None):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import argparse
    import torch
    import workloads as W
    from . import dalia as D

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("config", nargs="?", default="c1", choices=("c1", "c2", "c1_poisson"))
    ap.add_argument("--batch", type=int, default=0,
                    help="instances per pass (0: 2 dim + 1 for c1, 31 for c2)")
    ap.add_argument("--tiles", default=os.path.join(root, "paper_2507_06938_amd",
                                                    "tiles_gfx950.txt"))
    args = ap.parse_args(argv)
    poisson = args.config == "c1_poisson"
    wl = (W.config2() if args.config == "c2" else
          W.config1(likelihood="poisson" if poisson else "gaussian"))
    d = wl.dim_theta
    B = args.batch or (31 if args.config == "c2" else 2 * d + 1)
    model = D.Model.from_workload(wl)
    # counts: every instance's inner Newton search starts from its previous
    # mode (the stencil points of consecutive passes are h apart)
    ws = D.Workspace([model] * B, graph=True, warm_start=poisson)
    ws.autotune(args.tiles)
    fobj_hessian(ws, wl.theta)  # warm-up (graph capture)
    t0 = time.perf_counter()
    H, f0, vals = fobj_hessian(ws, wl.theta)
    t = time.perf_counter() - t0
    ev = np.linalg.eigvalsh(H)
    out = {"workload": wl.name, "dim_theta": d, "points": int(vals.size), "batch": B,
           "passes": int(-(-vals.size // B)), "s_per_hessian": t,
           "evals_per_s": vals.size / t, "f": float(f0),
           "hessian": H.tolist(), "eigenvalues": ev.tolist(),
           "negative_definite": bool(ev.max() < 0)}
    if poisson:
        out["newton_steps_last_pass"] = ws.newton_steps().tolist()
    if out["negative_definite"]:
        out["gaussian_marginal_sd"] = marginal_sd(H).tolist()
        A, sp, sm, sv = fobj_skew(ws, wl.theta, H, f0)
        out["skew_points"] = int(sv.size)
        if sp is not None:
            up, dn = skew_sd(A, sp, sm)
            out.update(skew_scale_plus=sp.tolist(), skew_scale_minus=sm.tolist(),
                       skew_sd_upper=up.tolist(), skew_sd_lower=dn.tolist())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
