"""Batched f_obj throughput: a central-difference gradient of the trivariate
30x30, nt = 48 model (31 theta points, Eq. 10) and the uneven 64-instance
mix, each as batched, graph-replayed workspaces in FP64 and mixed precision.

    python -m paper_2507_06938_amd.batch_study [--skip-uneven] [--skip-fd]

The uneven mix needs more device memory than one GPU holds at once, so the
library's planner (dl_plan_waves: first fit, largest first) splits it into
waves of at most --mem-gb of workspace each; a wave is one workspace of
uneven instances evaluated together.  Prints one
JSON document: evals/s of every configuration, the sequential single-
instance rate for comparison, device bytes, and whether every evaluation
reported positive-definite factors.
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
    ap.add_argument("--mem-gb", type=float, default=240.0)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--skip-uneven", action="store_true")
    ap.add_argument("--skip-fd", action="store_true")
    ap.add_argument("--order", choices=("one-sided", "two-sided"), default="one-sided",
                    help="elimination order of every workspace (two-sided: the two "
                         "halves of the time domain concurrently toward a middle block)")
    ap.add_argument("--tiles", default=os.path.join(root, "paper_2507_06938_amd",
                                                    "tiles_gfx950.txt"))
    args = ap.parse_args(argv)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    out = {}
    if not args.skip_fd:
        wl = W.config2()
        model = D.Model.from_workload(wl)
        h = 1e-3
        d = wl.dim_theta
        pts = np.repeat(wl.theta[None], 2 * d + 1, axis=0)
        for i in range(d):
            pts[1 + 2 * i, i] += h
            pts[2 + 2 * i, i] -= h
        th = torch.tensor(pts, dtype=torch.float64, device="cuda")
        res = {"workload": wl.name, "points": 2 * d + 1, "order": args.order}
        two = args.order == "two-sided"
        single = D.Workspace(model, two_sided=two, fold_inverse=True)
        single.autotune(args.tiles)
        t1 = timed(lambda: single.fobj(th[:1]), args.reps)
        res["single_fp64_evals_per_s"] = 1.0 / t1
        del single
        torch.cuda.empty_cache()
        for mixed in (False, True):
            ws = D.Workspace([model] * (2 * d + 1), graph=True, mixed=mixed, two_sided=two)
            ws.autotune(args.tiles)
            t = timed(lambda: ws.fobj(th), args.reps)
            f, parts, info = ws.fobj(th)
            torch.cuda.synchronize()
            key = "mixed" if mixed else "fp64"
            res[key] = {"s_per_gradient": t, "evals_per_s": (2 * d + 1) / t,
                        "speedup_vs_single_fp64": (2 * d + 1) / t * t1,
                        "device_gb": ws.nbytes / 1e9,
                        "all_spd": bool((info == 0).all().item()),
                        "f0": float(f[0].item())}
            print(key, json.dumps(res[key]), file=sys.stderr, flush=True)
            del ws
            torch.cuda.empty_cache()
        out["fd_gradient_c2"] = res

    if not args.skip_uneven:
        wls = [W.uneven_instance(k) for k in range(64)]
        models = [D.Model.from_workload(w) for w in wls]
        res = {"instances": 64}
        for mixed in (False, True):
            # the library's planner: first fit, largest first, within the budget
            waves = D.plan_waves(models, int(args.mem_gb * 1e9), graph=True, mixed=mixed,
                                 two_sided=args.order == "two-sided")
            total_t, ok, gb = 0.0, True, []
            for wave in waves:
                ws = D.Workspace([models[k] for k in wave], graph=True, mixed=mixed,
                                 two_sided=args.order == "two-sided")
                ws.autotune(args.tiles)
                th = np.concatenate([wls[k].theta for k in wave])
                t = timed(lambda: ws.fobj(th), args.reps)
                f, parts, info = ws.fobj(th)
                torch.cuda.synchronize()
                ok = ok and bool((info == 0).all().item())
                total_t += t
                gb.append(ws.nbytes / 1e9)
                print(("mixed" if mixed else "fp64"), "wave", len(wave), "instances",
                      f"{t:.3f} s", f"{ws.nbytes / 1e9:.1f} GB", file=sys.stderr, flush=True)
                del ws
                torch.cuda.empty_cache()
            res["mixed" if mixed else "fp64"] = {
                "waves": [len(w) for w in waves], "wave_gb": gb, "s_all": total_t,
                "evals_per_s": 64 / total_t, "all_spd": ok}
        out["uneven_64"] = res
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
