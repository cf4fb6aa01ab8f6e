"""Mode-search study (Eq. 9): plain batched finite-difference BFGS against the
surrogate-guided variant, from seeded starts theta_0 = theta* + 0.25 z.

    python -m paper_2507_06938_amd.opt_study --nx 12 --nt 12 --runs 16
    python -m paper_2507_06938_amd.opt_study --config2 --runs 3
    python -m paper_2507_06938_amd.opt_study --config2 --ref-in ref.json --methods mixed

``--config2`` takes the production trivariate model (30 x 30 mesh, nt = 48,
b = 2700, 31-point gradients) instead of the generator at --nx/--nt, and
``--config1`` the production univariate mesh (45 x 45, nt = 100); with
``--likelihood poisson`` the responses are counts.

theta* and F* = -f_obj(theta*) come from a reference FD-BFGS run started at
the generator's theta and driven to a small gradient.  Each method then runs
from every start until |F - F*| <= rtol |F*| (or its iteration cap), and the
study reports exact f_obj evaluations and wall time per run.  Methods: ``fd``
(FD-BFGS on FP64 evaluations), ``surrogate`` (surrogate-guided BFGS) and
``mixed`` (FD-BFGS on mixed-precision evaluations -- FP32 off-diagonal blocks,
FP64 diagonal blocks and refined mean -- finished on FP64 ones; the target is
always tested on FP64 values).  Every f_obj
value comes from the batched GPU evaluator; the surrogate network is trained
by the library's MLP kernels.  Prints one JSON document.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch


def main(argv=None):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import workloads as W
    from . import dalia as D
    from . import optimize as O

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--nx", type=int, default=12)
    ap.add_argument("--nt", type=int, default=12)
    ap.add_argument("--nv", type=int, default=3)
    ap.add_argument("--nr", type=int, default=2)
    ap.add_argument("--m-per", type=int, default=0,
                    help="observations (0: nv * nt * nx^2, one per node and step)")
    ap.add_argument("--runs", type=int, default=16)
    ap.add_argument("--scale", type=float, default=0.25)
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--train-steps", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--config2", action="store_true",
                    help="the production trivariate model (30x30, nt = 48)")
    ap.add_argument("--config1", action="store_true",
                    help="the production univariate mesh (45x45, nt = 100)")
    ap.add_argument("--likelihood", choices=("gaussian", "poisson"), default="gaussian",
                    help="responses: Gaussian, or counts (inner Newton search, "
                         "warm-started by the evaluator)")
    ap.add_argument("--ref-out", default=None,
                    help="write theta* and F* of the reference run to this JSON file")
    ap.add_argument("--ref-in", default=None,
                    help="take theta* and F* from a file written by --ref-out "
                         "instead of running the reference")
    ap.add_argument("--first-run", type=int, default=0,
                    help="index of the first seeded start (starts are drawn in order)")
    ap.add_argument("--progress-evals", type=int, default=500,
                    help="print a progress line every this many exact evaluations")
    ap.add_argument("--methods", default="fd,surrogate",
                    help="comma-separated subset of fd, surrogate, mixed")
    ap.add_argument("--fp64-batch", type=int, default=8,
                    help="instances of the FP64 evaluator when only the mixed method "
                         "runs and theta* is read from --ref-in (its target checks and "
                         "finishing gradients then go through it in chunks)")
    args = ap.parse_args(argv)
    methods = [m.strip() for m in args.methods.split(",") if m.strip()]
    if not methods or any(m not in ("fd", "surrogate", "mixed") for m in methods):
        ap.error("--methods takes a comma-separated subset of fd, surrogate, mixed")

    if args.config2:
        wl = W.config2(seed=args.seed, likelihood=args.likelihood)
    elif args.config1:
        wl = W.config1(seed=args.seed, likelihood=args.likelihood)
    else:
        m_per = args.m_per or args.nv * args.nt * args.nx * args.nx
        wl = W.scaled(f"opt_{args.nv}v_{args.nx}x{args.nx}_nt{args.nt}", args.nx, args.nt,
                      args.nv, args.nr, m_per, seed=args.seed, likelihood=args.likelihood)
    model = D.Model.from_workload(wl)
    d = wl.dim_theta
    B = 2 * d + 1

    class Logged(O.Evaluator):
        """The batched evaluator with a progress line on stderr."""
        mark = 0

        def __call__(self, thetas):
            v = super().__call__(thetas)
            if self.count - self.mark >= args.progress_evals:
                self.mark = self.count
                best = min(self.archive_f) if self.archive_f else float("nan")
                print(f"  exact evaluations {self.count}, best F {best:.10f}",
                      file=sys.stderr, flush=True)
            return v

    # the FP64 evaluator runs the reference and the fd / surrogate methods at
    # full gradient batch; for the mixed method alone it only checks targets
    # and finishes, at a smaller batch (the two workspaces share HBM)
    full64 = "fd" in methods or "surrogate" in methods or not args.ref_in
    ev = Logged(model, B if full64 else min(B, args.fp64_batch), graph=True)
    evm = Logged(model, B, graph=True, mixed=True) if "mixed" in methods else None

    # reference optimum
    if args.ref_in:
        with open(args.ref_in) as fh:
            saved = json.load(fh)
        assert saved["workload"] == wl.name
        theta_star, F_star = np.asarray(saved["theta_star"]), float(saved["F_star"])
        ref_info = saved["reference"]
    else:
        t0 = time.perf_counter()
        ref = O.fd_bfgs(ev, wl.theta, h=1e-3, ftol=0.0, gtol=1e-5, max_iter=400)
        theta_star, F_star = ref.theta[-1], ref.f[-1]
        t_ref = time.perf_counter() - t0
        ref_info = {"iters": len(ref.f) - 1, "exact_evals": ref.exact_evals[-1],
                    "wall_s": t_ref, "F_start": float(ref.f[0])}
        print(f"reference: F* = {F_star:.12f}, {len(ref.f) - 1} iterations, {t_ref:.1f} s",
              file=sys.stderr, flush=True)
        if args.ref_out:
            with open(args.ref_out, "w") as fh:
                json.dump({"workload": wl.name, "theta_star": list(map(float, theta_star)),
                           "F_star": float(F_star), "reference": ref_info}, fh)

    def fresh():
        for e in (ev, evm):
            if e is None:
                continue
            e.count = 0
            e.mark = 0
            e.archive_x.clear()
            e.archive_f.clear()

    runs = []
    rng = np.random.default_rng(12345 + args.seed)
    starts = [theta_star + args.scale * rng.standard_normal(d)
              for _ in range(args.first_run + args.runs)][args.first_run:]
    for k, th0 in enumerate(starts, start=args.first_run):
        row = {"run": k}
        if "fd" in methods:
            fresh()
            t0 = time.perf_counter()
            tr = O.fd_bfgs(ev, th0, h=1e-3, ftol=0.0, gtol=0.0, max_iter=args.max_iter,
                           f_target=F_star, target_rtol=args.rtol)
            torch.cuda.synchronize()
            row["fd"] = {"exact_evals": tr.exact_evals[-1],
                         "wall_s": time.perf_counter() - t0,
                         "F": float(tr.f[-1]),
                         "iters": len(tr.f) - 1,
                         "reached": bool(abs(tr.f[-1] - F_star) <= args.rtol * abs(F_star)),
                         "rel_gap": float(abs(tr.f[-1] - F_star) / abs(F_star))}
        if "surrogate" in methods:
            fresh()
            sur = O.Surrogate(d, hidden=(256, 256, 256),
                              max_batch=(args.max_iter + 2) * 3 * B, seed=k)
            t0 = time.perf_counter()
            tr = O.surrogate_bfgs(ev, th0, sur, h=1e-3, ftol=0.0, gtol=0.0,
                                  max_iter=args.max_iter, f_target=F_star,
                                  target_rtol=args.rtol, train_steps=args.train_steps)
            torch.cuda.synchronize()
            row["surrogate"] = {
                "exact_evals": tr.exact_evals[-1], "F": float(tr.f[-1]),
                "wall_s": time.perf_counter() - t0,
                "iters": len(tr.f) - 1,
                "surrogate_steps": tr.kind.count("surrogate"),
                "fd_steps": tr.kind.count("fd"),
                "reached": bool(abs(tr.f[-1] - F_star) <= args.rtol * abs(F_star)),
                "rel_gap": float(abs(tr.f[-1] - F_star) / abs(F_star))}
        if "mixed" in methods:
            fresh()
            t0 = time.perf_counter()
            tr = O.mixed_fd_bfgs(evm, ev, th0, h=1e-3, ftol=0.0, gtol=0.0,
                                 max_iter=args.max_iter, f_target=F_star,
                                 target_rtol=args.rtol)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            F64 = float(ev(np.asarray(tr.theta[-1])[None])[0])
            row["mixed"] = {"exact_evals": evm.count + ev.count - 1,
                            "mixed_evals": evm.count, "fp64_evals": ev.count - 1,
                            "mixed_not_spd": evm.count - len(evm.archive_f),
                            "wall_s": wall, "F_fp64": F64,
                            "iters": len(tr.f) - 1,
                            "mixed_steps": tr.kind.count("mixed"),
                            "fp64_steps": tr.kind.count("fd"),
                            "reached": bool(abs(F64 - F_star) <= args.rtol * abs(F_star)),
                            "rel_gap": float(abs(F64 - F_star) / abs(F_star))}
        runs.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)

    def summ(key):
        ok = [r[key] for r in runs if r[key]["reached"]]
        return {"reached": len(ok), "of": len(runs),
                "median_exact_evals": float(np.median([r["exact_evals"] for r in ok])) if ok else None,
                "median_wall_s": float(np.median([r["wall_s"] for r in ok])) if ok else None,
                "mean_exact_evals": float(np.mean([r["exact_evals"] for r in ok])) if ok else None}
    out = {"workload": wl.name, "N": wl.N, "b": wl.b, "dim_theta": d, "batch": B,
           "F_star": float(F_star), "theta_star": list(map(float, theta_star)),
           "reference": ref_info,
           "rtol": args.rtol, "start_scale": args.scale, "runs": runs}
    for m, key in (("fd", "fd_bfgs"), ("surrogate", "surrogate_bfgs"),
                   ("mixed", "mixed_fd_bfgs")):
        if m in methods:
            out[key] = summ(m)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
