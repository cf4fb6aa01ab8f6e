"""f_obj for Poisson counts (Laplace approximation with a damped Newton
search for the inner mode) on the production univariate mesh (45 x 45,
nt = 100, 4 fixed effects, m = 200000), against the Gaussian f_obj of the
same mesh: time per evaluation, Newton steps, time per Newton step, and a
batched central-difference gradient (2 dim + 1 = 7 points, Eq. 10) whose
instances converge at their own step counts, cold and warm-started (the next
gradient of an optimiser, 0.01 away, each Newton search starting from the
previous gradient's modes).

    python -m paper_2507_06938_amd.laplace_study [--reps 3] [--poisson-only]

Prints one JSON document.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def main(argv=None):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import numpy as np
    import torch
    import workloads as W
    from . import dalia as D

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--poisson-only", action="store_true",
                    help="only the single Poisson evaluation (for kernel profiles)")
    ap.add_argument("--tiles", default=os.path.join(root, "paper_2507_06938_amd",
                                                    "tiles_gfx950.txt"))
    args = ap.parse_args(argv)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.reps

    out = {}
    kw = dict(two_sided=True, fold_inverse=True)
    for lik in (("poisson",) if args.poisson_only else ("gaussian", "poisson")):
        wl = W.make_univariate(f"c1_{lik}", 45, 100, 4, 200_000, seed=0, likelihood=lik)
        model = D.Model.from_workload(wl)
        ws = D.Workspace(model, **kw)
        ws.autotune(args.tiles)
        th = torch.tensor(wl.theta[None], dtype=torch.float64, device="cuda")
        t = timed(lambda: ws.fobj(th))
        f, parts, info = ws.fobj(th)
        torch.cuda.synchronize()
        res = {"workload": wl.name, "dim_theta": wl.dim_theta, "ms_per_fobj": 1e3 * t,
               "f": float(f[0].item()), "spd": bool((info == 0).all().item()),
               "rel_residual": float(parts[0, 7].item())}
        if lik == "poisson":
            steps = int(ws.newton_steps()[0])
            res["newton_steps"] = steps
            # each step: weights, assembly, factor and solve of Q_c, trials;
            # plus Q_p once and Q_c at the mode
            res["ms_per_newton_step"] = 1e3 * t / (steps + 1)
        print(lik, json.dumps(res), file=sys.stderr, flush=True)
        out[lik] = res
        del ws
        torch.cuda.empty_cache()
        if lik == "poisson" and not args.poisson_only:
            d = wl.dim_theta
            h = 1e-3
            pts = np.repeat(wl.theta[None], 2 * d + 1, axis=0)
            for i in range(d):
                pts[1 + 2 * i, i] += h
                pts[2 + 2 * i, i] -= h
            thb = torch.tensor(pts, dtype=torch.float64, device="cuda")
            wsb = D.Workspace([model] * (2 * d + 1), **kw)
            wsb.autotune(args.tiles)
            tb = timed(lambda: wsb.fobj(thb))
            fb, _, ib = wsb.fobj(thb)
            torch.cuda.synchronize()
            out["poisson_fd_gradient"] = {
                "points": 2 * d + 1, "s_per_gradient": tb, "evals_per_s": (2 * d + 1) / tb,
                "newton_steps": wsb.newton_steps().tolist(),
                "all_spd": bool((ib == 0).all().item()),
                "gradient": ((fb[1::2] - fb[2::2]) / (2 * h)).cpu().numpy().tolist()}
            print("fd", json.dumps(out["poisson_fd_gradient"]), file=sys.stderr, flush=True)
            del wsb
            torch.cuda.empty_cache()
            # the next gradient of an optimiser, 0.01 away, with each instance's
            # Newton search started from its mode of the previous gradient
            wsw = D.Workspace([model] * (2 * d + 1), warm_start=True, **kw)
            wsw.autotune(args.tiles)
            wsw.fobj(thb)
            torch.cuda.synchronize()
            shift = torch.full_like(thb, 0.0)
            shift[:, 0] = 0.01
            t0 = time.perf_counter()
            fw, _, iw = wsw.fobj(thb + shift)
            torch.cuda.synchronize()
            tw = time.perf_counter() - t0
            out["poisson_fd_gradient_warm"] = {
                "points": 2 * d + 1, "s_per_gradient": tw, "evals_per_s": (2 * d + 1) / tw,
                "newton_steps": wsw.newton_steps().tolist(),
                "all_spd": bool((iw == 0).all().item())}
            print("fd warm", json.dumps(out["poisson_fd_gradient_warm"]), file=sys.stderr,
                  flush=True)
            del wsw
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
