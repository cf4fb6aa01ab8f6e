#!/usr/bin/env python3
"""f_obj throughput on one MI355X.

One step = one full pass of the evaluation path for one hyperparameter
vector of the production univariate workload (45x45 mesh, b = 2025,
nt = 100, 4 fixed effects, 200,000 observations): theta -> coefficients,
assembly of Q_p and Q_c into dense BTA blocks, BTA Cholesky of both,
log-determinants, forward/backward solve for the conditional mean, the
quadratic forms and f_obj, then the selected inversion of Q_c for all
marginal variances.  By default the time domain is split into two
partitions eliminated concurrently toward a middle block (``--order
two-sided``; ``one-sided`` sweeps the time steps forward only).  Inputs are
seeded and synthetic and already resident on the device when the timed
region starts.  Single evaluations form the diagonal blocks' inverses inside
the launches of their factorisation (the batched gradient keeps the
recursive GEMM inversion, which is faster for many blocks at once).

Prints one JSON line.  Besides the metric it reports the BTA Cholesky
TFLOP/s of Q_c alone, the log-determinant error against the FP64 CPU oracle
(stored values written by tests/golden/make_golden.py), the live roofline of
the dominant kernel (HIP events around its launches during the timed steps)
and the CPU oracle timed on a bounded sample of the same workload.  GEMM
tiles are the measured choices of the library's autotuner (cache file
paper_2507_06938_amd/tiles_gfx950.txt; missing shapes are timed and added).
Three further measurements of the same mesh are extra fields of the line:
the 9-point central-difference gradient as one batched, graph-replayed
evaluation, f_obj in mixed precision with its errors, and f_obj with
Poisson counts in place of the Gaussian responses (inner damped Newton and
Laplace approximation) with its errors against stored oracle values.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("f_obj evals/s + BTA Cholesky TFLOP/s (ns=2000,nt=100); "
          "logdet rel err vs FP64")
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def fac_flops(n, b, a):
    """Algorithmic FLOPs of one BTA Cholesky (LAPACK counts: POTRF b^3/3,
    TRSM m n^2, SYRK n^2 k, GEMM 2mnk)."""
    return (n * (b ** 3 / 3 + a * b * b + a * a * b)
            + (n - 1) * (2 * b ** 3 + 2 * a * b * b) + a ** 3 / 3)


# HBM bytes per algorithmic FLOP of the FP64 tile GEMM on the launch shapes
# of each category, from rocprofv3 FETCH_SIZE and WRITE_SIZE runs of the GEMM
# microbenchmark (64-wide tiles, counters scaled by a plain device copy;
# profiles/gemm_block_products_traffic.md):
#   trsm    [B;R] G^T, 2112 x 2048 x 2048, k < col + 64: 610.6 + 34.6 MB / 8.858 GFLOP
#   update  SYRK lower 2048^2, K 2048:                  174.6 + 16.8 MB / 8.590 GFLOP
#   selinv  per recursion step: W = [B;R] G (as trsm), Y = -X W (NN 2112 x 2048 x 2112,
#           432.6 + 34.6 MB / 18.27 GFLOP), X_tt -= Y^T W (as update), G^T G (lower,
#           k >= row, 224.5 + 16.8 MB / 5.727 GFLOP): 1.545 GB / 41.45 GFLOP
#   other   NN 2048^3: 307.1 + 33.6 MB / 17.18 GFLOP
GEMM_BYTES_PER_FLOP = {"trsm": 645.2e6 / 8.858e9, "update": 191.4e6 / 8.590e9,
                       "selinv": 1.545e9 / 41.45e9, "other": 340.7e6 / 17.18e9}


def cpu_model():
    """The host CPU's model name and logical CPU count."""
    name = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name, os.cpu_count()


def cpu_baseline(var_samples: int = 8, model: str = "separable"):
    """The CPU oracle on the benchmark's own workload: one full-size f_obj
    (RCM + LAPACK banded Cholesky of Q_p and Q_c, the solve for mu, Eq. 8),
    measured, plus var_samples unit-vector solves with the factor of Q_c for
    single marginal variances, scaled to all N diagonal entries (the oracle
    has no selected inversion)."""
    import numpy as np
    from threadpoolctl import threadpool_info
    import workloads as W
    from oracle import fobj as OF
    wl = W.config1(model=model)
    t0 = time.perf_counter()
    p = OF.fobj_parts(wl, wl.theta, method="banded", return_factors=True)
    t1 = time.perf_counter()
    idx = np.random.default_rng(0).choice(wl.N, var_samples, replace=False)
    p["Fc"].inv_diag(idx, chunk=1)
    t2 = time.perf_counter()
    t_fobj = t1 - t0
    t_var = (t2 - t1) / var_samples * wl.N
    threads = max((i.get("num_threads", 1) for i in threadpool_info()),
                  default=1)
    name, ncpu = cpu_model()
    return {
        "value": 1.0 / (t_fobj + t_var), "unit": "evals/s", "cores": threads,
        "kind": "oracle", "cpu_model": name, "logical_cpus": ncpu,
        "fobj_only_evals_per_s": 1.0 / t_fobj, "fobj_seconds_measured": t_fobj,
        "f": p["f"],
        "sample": (f"oracle (RCM + LAPACK banded Cholesky) f_obj of {wl.name} at full "
                   f"size, measured once ({t_fobj:.1f} s); all N={wl.N} marginal "
                   f"variances extrapolated from {var_samples} unit-vector solves "
                   f"({t2 - t1:.2f} s) with the same factor"),
    }


def _events_ms(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def fd_batch(D, W, wl, model, single_ms, tiles, two_sided=False, dag=False):
    """The 2 dim(theta) + 1 = 9 central-difference points of one gradient
    (Eq. 10, h = 1e-3) as one batched, graph-replayed evaluation."""
    import numpy as np
    import torch
    h = 1e-3
    d = wl.dim_theta
    pts = np.repeat(wl.theta[None], 2 * d + 1, axis=0)
    for i in range(d):
        pts[1 + 2 * i, i] += h
        pts[2 + 2 * i, i] -= h
    th = torch.tensor(pts, dtype=torch.float64, device="cuda")
    ws = D.Workspace([model] * (2 * d + 1), graph=True, two_sided=two_sided, dag=dag)
    if tiles:
        ws.autotune(tiles)
    ms = _events_ms(torch, lambda: ws.fobj(th), 3)
    f, _, info = ws.fobj(th)
    torch.cuda.synchronize()
    grad = ((f[1::2] - f[2::2]) / (2 * h)).cpu().numpy().tolist()
    ok = bool((info == 0).all().item())
    del ws
    torch.cuda.empty_cache()
    return {"points": 2 * d + 1, "ms_per_gradient": ms,
            "evals_per_s": (2 * d + 1) * 1000.0 / ms,
            "speedup_vs_sequential": (2 * d + 1) * single_ms / ms,
            "gradient": grad, "all_spd": ok}


def poisson(D, W, tiles, two_sided=False):
    """f_obj of the same mesh with Poisson counts (inner damped Newton for
    the mode, Laplace approximation), against the stored oracle values."""
    import torch
    wl = W.config1(likelihood="poisson")
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, two_sided=two_sided, fold_inverse=True)
    if tiles:
        ws.autotune(tiles)
    th = torch.tensor(wl.theta, dtype=torch.float64, device="cuda")
    ms = _events_ms(torch, lambda: ws.fobj(th), 2)
    f, parts, info = ws.fobj(th)
    torch.cuda.synchronize()
    p = parts.cpu().numpy()[0]
    out = {"workload": wl.name, "evals_per_s": 1000.0 / ms, "ms": ms,
           "newton_steps": int(ws.newton_steps()[0]), "f": float(p[0]),
           "rel_gradient_at_mode": float(p[7]),
           "spd": bool((info == 0).all().item())}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                        "c1_poisson_golden.json")
    if os.path.exists(path):
        g = json.load(open(path))
        scale = abs(g["logdet_p"]) + abs(g["logdet_c"])
        out["err_vs_fp64_oracle"] = {"f_rel_scale": abs(p[0] - g["f"]) / scale,
                                     "logdet_c_rel": abs(p[2] - g["logdet_c"]) / abs(g["logdet_c"]),
                                     "oracle_newton_steps": g["newton_steps"]}
    del ws
    torch.cuda.empty_cache()
    return out


def mixed(D, wl, model, errors, tiles, two_sided=False, dag=False):
    """f_obj with FP32 off-diagonal blocks (FP64 diagonal blocks, tip and
    refinement of the mean) at the same theta."""
    import torch
    ws = D.Workspace(model, mixed=True, two_sided=two_sided, fold_inverse=not dag, dag=dag)
    if tiles:
        ws.autotune(tiles)
    th = torch.tensor(wl.theta, dtype=torch.float64, device="cuda")
    ms = _events_ms(torch, lambda: ws.fobj(th), 3)
    f, parts, info = ws.fobj(th)
    torch.cuda.synchronize()
    p = parts.cpu().numpy()[0]
    # where one evaluation's time goes: summed launch durations (HIP events
    # around each launch) by operation category and by kernel
    split = {}
    for by_kernel in (False, True):
        ws.profile_begin(D.CATEGORIES, max_launches=40000, by_kernel=by_kernel)
        ws.fobj(th)
        torch.cuda.synchronize()
        split["by_kernel" if by_kernel else "by_category"] = {
            k: round(v["ms"], 3) for k, v in ws.profile_end().items()}
    del ws
    torch.cuda.empty_cache()
    return {"evals_per_s": 1000.0 / ms, "ms": ms,
            "err_vs_fp64_oracle": errors(p),
            "refined_mean_rel_residual": float(p[7]),
            "launch_ms": split}


def gemm_roofline(prof, steps):
    """Roofline of the dominant kernel, the FP64 MFMA tile GEMM, from the
    HIP events around its launches in `steps` bracketed timed steps
    (algorithmic LAPACK flop counts of the products it ran; the split-k
    reductions, a separate kernel, are reported beside it)."""
    gk = prof.get("k_gemm_tasks", {"ms": 0.0, "launches": 0, "flops": 0.0})
    red = prof.get("k_gemm_reduce", {"ms": 0.0, "launches": 0})
    achieved = gk["flops"] / (gk["ms"] * 1e-3) / 1e12 if gk["ms"] else 0.0
    return {
        "kernel": "k_gemm_tasks (FP64 MFMA 16x16x4 tile GEMM, 64- and 128-wide tiles)",
        "bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
        "traffic": None,
        "launches": gk["launches"],
        "avg_launch_us": 1000.0 * gk["ms"] / max(1, gk["launches"]),
        "alg_flops_per_launch": gk["flops"] / max(1, gk["launches"]),
        "split_reduce_ms_per_step": red["ms"] / max(1, steps),
    }


def check_timed_step(g, p, info, var, mu):
    """The timed step's f_obj, log-determinants, quadratic forms, mean and
    marginal variances against the stored oracle values `g` (None: no stored
    values), with the parity tolerances of the tests: log-determinants
    1e-10 relative, f 1e-10 (|log|Q_p|| + |log|Q_c||), quadratic forms 1e-9
    relative, mean 1e-9 max|mu|, variances 1e-9 relative."""
    import numpy as np
    if g is None:
        return None
    scale = abs(g["logdet_p"]) + abs(g["logdet_c"])
    mu_s = mu[np.asarray(g["mu_index_bta"])]
    mu_want = np.asarray(g["mu"])
    v_s = var[np.asarray(g["var_index_bta"])]
    v_want = np.asarray(g["var"])
    e = {"logdet_p_rel": abs(p[1] - g["logdet_p"]) / abs(g["logdet_p"]),
         "logdet_c_rel": abs(p[2] - g["logdet_c"]) / abs(g["logdet_c"]),
         "f_abs": abs(p[0] - g["f"]),
         "f_rel_scale": abs(p[0] - g["f"]) / scale,
         "quad_p_rel": abs(p[3] - g["quad_p"]) / abs(g["quad_p"]),
         "quad_obs_rel": abs(p[4] - g["quad_obs"]) / abs(g["quad_obs"]),
         "mu_rel_max": float(np.max(np.abs(mu_s - mu_want)) / np.max(np.abs(mu_want))),
         "var_rel_max": float(np.max(np.abs(v_s - v_want) / v_want)),
         "mu_positions": int(mu_s.size), "var_positions": int(v_s.size)}
    e["ok"] = bool(info.tolist() == [[0, 0]] and e["logdet_p_rel"] <= 1e-10
                   and e["logdet_c_rel"] <= 1e-10 and e["f_rel_scale"] <= 1e-10
                   and e["quad_p_rel"] <= 1e-9 and e["quad_obs_rel"] <= 1e-9
                   and e["mu_rel_max"] <= 1e-9 and e["var_rel_max"] <= 1e-9
                   and bool(np.all(np.isfinite(var))) and bool(np.all(var > 0)))
    return e


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FD-batch and mixed-precision measurements")
    ap.add_argument("--roofline-only", action="store_true",
                    help="run only the warmup and timed steps and print their "
                         "line (the launch mix a kernel profiler then sees is "
                         "the timed region's)")
    ap.add_argument("--model", choices=("separable", "diffusion"),
                    default="separable",
                    help="model family of the workload (the headline is the "
                         "separable one; 'diffusion' times the non-separable "
                         "space-time model on the same mesh and data)")
    ap.add_argument("--order", choices=("one-sided", "two-sided"),
                    default="two-sided",
                    help="elimination order: time steps forward only, or the "
                         "two halves of the time domain concurrently toward "
                         "a middle block (two time-domain partitions)")
    ap.add_argument("--cpu-only", action="store_true",
                    help="only run the CPU oracle leg (full-size f_obj on the host, "
                         "no GPU) and print it")
    ap.add_argument("--diag-factor", choices=("panel", "dag"), default="dag",
                    help="diagonal blocks factored by one launch per 64-column "
                         "panel, or by one persistent tile-task launch per "
                         "elimination step")
    ap.add_argument("--tiles", default=os.path.join(
        ROOT, "paper_2507_06938_amd", "tiles_gfx950.txt"),
        help="autotuner cache ('' disables tuning: default tiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the "
              "evaluation path is built for a single GPU and does not shard "
              "over several.", file=sys.stderr)
        sys.exit(2)

    if args.cpu_only:
        print(json.dumps(cpu_baseline(model=args.model)), flush=True)
        return

    import torch
    from paper_2507_06938_amd import dalia as D
    if not os.path.exists(D.LIB_PATH):
        from paper_2507_06938_amd import build as B
        B.build(verbose=False)
    import workloads as W

    wl = W.config1(model=args.model)
    model = D.Model.from_workload(wl)
    two_sided = args.order == "two-sided"
    dag = args.diag_factor == "dag"
    ws = D.Workspace(model, selinv=True, two_sided=two_sided, fold_inverse=not dag, dag=dag)
    tiles = ws.autotune(args.tiles) if args.tiles else None
    dev = torch.device("cuda")
    theta = torch.tensor(wl.theta, dtype=torch.float64, device=dev)
    f = torch.empty(1, dtype=torch.float64, device=dev)
    parts = torch.empty((1, 8), dtype=torch.float64, device=dev)
    info = torch.empty((1, 2), dtype=torch.int64, device=dev)
    var = torch.empty(model.N, dtype=torch.float64, device=dev)

    def step():
        # f_obj and all marginal variances; the solve overlaps the selected
        # inversion on a second stream
        ws.fobj_selinv(theta, out=(f, parts, info, var))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region; in its last step the FP64 MFMA GEMM kernel's launches
    # are bracketed by HIP events on the stream they run on (the diagonal
    # blocks' launches, other kernels, are not).  The steps are identical;
    # bracketing every step would add about 14 ms of event packets per step
    # to the timed region.  The event pool is created before timing.
    gemm_cats = ("panel_trsm", "trtri", "trsm", "update", "selinv")
    ws.profile_begin(gemm_cats, max_launches=40000, by_kernel=True)
    ws.profile_enable(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        if i == args.steps - 1:
            ws.profile_enable(True)
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ws.profile_end()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    # the last timed step's own outputs (nothing has run since), checked
    # against the stored oracle values below
    timed_out = (parts.cpu().numpy()[0].copy(), info.cpu().numpy().copy(),
                 var.cpu().numpy().copy(), ws.mean().cpu().numpy())
    # untimed steps, one per category, recording the GEMM kernel's
    # algorithmic FLOPs in that category, for the modeled HBM traffic of the
    # dominant kernel
    fl = {}
    for c in gemm_cats:
        ws.profile_begin((c,), max_launches=40000, by_kernel=True)
        step()
        torch.cuda.synchronize()
        fl[c] = ws.profile_end().get("k_gemm_tasks", {}).get("flops", 0.0)
    model_bytes = (fl["trsm"] * GEMM_BYTES_PER_FLOP["trsm"]
                   + fl["update"] * GEMM_BYTES_PER_FLOP["update"]
                   + fl["selinv"] * GEMM_BYTES_PER_FLOP["selinv"]
                   + (fl["panel_trsm"] + fl["trtri"]) * GEMM_BYTES_PER_FLOP["other"])
    value = args.steps / (t1 - t0)
    roofline = gemm_roofline(prof, 1)
    roofline["steps_bracketed"] = 1
    if args.roofline_only:
        print(json.dumps({"metric": METRIC, "value": value, "unit": "evals/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": ms_per_step, "roofline": roofline,
                          "profile_by_kernel": prof}), flush=True)
        return

    # f_obj alone (no selected inversion), and the BTA Cholesky of Q_c
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        ws.fobj(theta, out=(f, parts, info))
    e1.record()
    torch.cuda.synchronize()
    fobj_ms = e0.elapsed_time(e1) / 3
    fac_ms = []
    for _ in range(3):
        ws.assemble(theta, D.DL_QC)
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record()
        ld, inf = ws.factor(D.DL_QC)
        a1.record()
        torch.cuda.synchronize()
        fac_ms.append(a0.elapsed_time(a1))
    fac_ms = sorted(fac_ms)[1]
    F = fac_flops(wl.nt, wl.b, wl.a)
    ws.fobj(theta, out=(f, parts, info))
    torch.cuda.synchronize()
    pr = parts.cpu().numpy()[0]

    golden_path = os.path.join(
        ROOT, "tests", "golden",
        "c1_golden.json" if args.model == "separable" else f"c1_{args.model}_golden.json")
    g = json.load(open(golden_path)) if os.path.exists(golden_path) else None

    def errors(p):
        if g is None:
            return None
        return {"logdet_p": abs(p[1] - g["logdet_p"]) / abs(g["logdet_p"]),
                "logdet_c": abs(p[2] - g["logdet_c"]) / abs(g["logdet_c"]),
                "f_abs": abs(p[0] - g["f"])}
    err = errors(pr)
    check = check_timed_step(g, *timed_out)
    launches = max(1, roofline["launches"])
    roofline["traffic"] = model_bytes / launches
    roofline["traffic_source"] = (
        "modeled, not counted on this process: HBM bytes per algorithmic FLOP measured by "
        "rocprofv3 FETCH_SIZE/WRITE_SIZE on the GEMM microbenchmark's launch shapes of each "
        "category (profiles/gemm_block_products_traffic.md), times this step's algorithmic "
        "FLOPs per category, per k_gemm_tasks launch")
    roofline["traffic_over_algorithmic_flops_bytes"] = {
        c: GEMM_BYTES_PER_FLOP[c] for c in GEMM_BYTES_PER_FLOP}

    out = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "ns": wl.ns, "nt": wl.nt,
                   "nb": wl.a, "m": wl.m, "b": wl.b, "N": wl.N,
                   "step": "fobj_eval + bta_selinv (all marginal variances)",
                   "order": args.order,
                   "block_inverse": ("inside the persistent tile-task launches" if dag
                                     else "inside the panel launches"),
                   "gemm_tiles": tiles},
        "fobj_only_evals_per_s": 1000.0 / fobj_ms,
        "bta_cholesky_tflops": F / (fac_ms * 1e-3) / 1e12,
        "bta_cholesky_ms": fac_ms,
        "logdet_rel_err_vs_fp64_oracle": err,
        "timed_step_vs_oracle": check,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    del ws
    torch.cuda.empty_cache()
    if not args.no_extras:
        # (the batch keeps the panel launches: with nine instances' blocks in
        # each persistent launch it measured 7.5 evals/s against 8.8)
        out["fd_gradient_batch"] = fd_batch(D, W, wl, model, fobj_ms, args.tiles,
                                            two_sided, dag=False)
        out["mixed_precision"] = mixed(D, wl, model, errors, args.tiles, two_sided, dag)
        if args.model == "separable":
            out["poisson_likelihood"] = poisson(D, W, args.tiles, two_sided)
    if not args.no_cpu_baseline:
        print("GPU legs done; timing the CPU oracle on the full-size workload",
              file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(model=args.model)
    print(json.dumps(out), flush=True)
    if check is not None and not check["ok"]:
        print("the timed step's outputs are outside the parity tolerances",
              file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
