"""Benchmark: one CSFMM evaluation per step on one MI355X.

Workload (the headline configuration): Poisson log kernel on the equiangular
cubed sphere with 256 x 256 cells per face (N = 393,216, same target and
source set, i = j omitted), field f = sum_{n=1..32} a_nm Y_nm with seeded
N(0, 1/(n+1)^2) coefficients minus its area mean, w = f A; theta = 0.7,
leaf <= 128, degree p (default 8) in the FP32 form (FP32 kernel evaluations,
FP64 geometry, interpolation and sums).  The plan (trees, lists) is built
once before timing; a step is one csfmm_eval: P2M, M2M, PP+PC, CP+CC, L2L,
L2P.  Inputs are resident in HBM before the timed region.

Prints one JSON line (see the repository's benchmark contract).
"""

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "N^2-equiv interactions/s per FMM eval at rel L2 err<=1e-5; p50/p99 latency"
UNIT = "N^2-equiv interactions/s"
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (published)
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector (published)
VALU_SLOTS_PER_S = 256 * 64 * 2.4e9  # 256 CUs x 64 lanes x 2.4 GHz

# Minimal FP32-form work per Poisson evaluation in the tile kernel:
# 3 sub, 1 mul + 2 fma (squared distance), 1 log2, 1 select, 1 fma.
FLOP_PER_EVAL = {"fp32": 3 + 1 + 4 + 1 + 2, "fp64": 3 + 1 + 4 + 1 + 2}
SLOTS_PER_EVAL_FP32 = 3 + 3 + 4 + 2 + 1  # log at quarter rate = 4 slots


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--E", type=int, default=256)
    ap.add_argument("--form", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def timed_evals(cs, torch, plan, W, out, steps, warmup):
    for _ in range(warmup):
        plan.eval(W, out=out)
    torch.cuda.synchronize()
    plan.timing(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        plan.eval(W, out=out)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    n, stage = plan.timing_read()
    plan.timing(False)
    return wall, lat, n, stage


def cpu_baseline(P, w, seconds):
    """The direct-sum oracle on the host cores, on a bounded sample of targets."""
    from oracle import direct, oracle_threads
    from workloads import config_subset
    n = P.shape[0]
    m = 256
    t = 0.0
    while True:
        S = config_subset(n, m, 2003)
        t0 = time.perf_counter()
        direct(1, P[S], P, w)
        t = time.perf_counter() - t0
        if t > seconds / 4 or m >= n:
            break
        m = min(n, int(m * max(2.0, 0.9 * seconds / 4 / max(t, 1e-3))))
    if t < seconds / 2 and m < n:
        m2 = min(n, int(m * seconds / max(t, 1e-3)))
        S = config_subset(n, m2, 2003)
        t0 = time.perf_counter()
        direct(1, P[S], P, w)
        t = time.perf_counter() - t0
        m = m2
    return {"value": m * n / t, "unit": UNIT, "cores": oracle_threads(), "kind": "oracle",
            "sample": "FP64 direct-sum oracle (C, OpenMP): %d seeded targets x all %d sources "
                      "in %.1f s; N^2-equiv rate = pairs/s" % (m, n, t),
            "host": platform.processor() or platform.machine()}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (--gpus 1); multi-GPU runs are not part of "
              "this build", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2508_13550_amd as cs
    from workloads import make_config, config_subset

    cfg = make_config(2, E=args.E)
    P, w = cfg["sources"], cfg["weights"]
    N = P.shape[0]
    dev = torch.device("cuda:0")
    T = torch.tensor(P, dtype=torch.float64, device=dev)
    W = torch.tensor(w, dtype=torch.float64, device=dev)
    theta, leaf = cfg["theta"], cfg["leaf"]

    results = {}
    for form in ("fp32", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = cs.Plan(T, None, kernel=cs.POISSON, p=args.p, theta=theta, leaf_size=leaf,
                       fp32=(form == "fp32"))
        torch.cuda.synchronize()
        plan_ms = 1e3 * (time.perf_counter() - t0)
        out = torch.empty(N, dtype=torch.float64, device=dev)
        steps = args.steps if form == args.form else max(5, args.steps // 5)
        wall, lat, n_t, stage = timed_evals(cs, torch, plan, W, out, steps, args.warmup)
        st = plan.stats()
        # accuracy on the seeded 4,096-target sample against the GPU FP64 direct sum
        S = config_subset(N, 4096, cfg["subset_seed"])
        idx = torch.tensor(S, device=dev)
        ref = cs.direct(T[idx].contiguous(), T, W, kernel=cs.POISSON)
        phi = out[idx]
        rel = float(torch.sqrt(torch.sum((phi - ref) ** 2) / torch.sum(ref ** 2)))
        mx = float(torch.max(torch.abs(phi - ref)) / torch.max(torch.abs(ref)))
        results[form] = dict(plan=plan, plan_ms=plan_ms, wall=wall, lat=lat, steps=steps,
                             stage={k: v / max(n_t, 1) for k, v in stage.items()}, stats=st,
                             rel=rel, max=mx)
        plan.close()
        del plan

    # GPU direct sum on the sample (same-device baseline)
    S = config_subset(N, 4096, cfg["subset_seed"])
    idx = torch.tensor(S, device=dev)
    Ts = T[idx].contiguous()
    direct_rate = {}
    for form in ("fp64", "fp32"):
        cs.direct(Ts, T, W, kernel=cs.POISSON, fp32=(form == "fp32"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            cs.direct(Ts, T, W, kernel=cs.POISSON, fp32=(form == "fp32"))
        torch.cuda.synchronize()
        direct_rate[form] = 3 * len(S) * N / (time.perf_counter() - t0)

    r = results[args.form]
    ms = 1e3 * r["wall"] / r["steps"]
    value = float(N) * N / (ms / 1e3)
    st = r["stats"]
    near_ms = r["stage"]["near"]
    evals_near = st["evals_pp"] + st["evals_pc"]
    fpe = FLOP_PER_EVAL[args.form]
    achieved = evals_near * fpe / (near_ms / 1e3) / 1e12
    peak = PEAK_FP32_TFLOPS if args.form == "fp32" else PEAK_FP64_TFLOPS
    roofline = {"bound": "alu", "kernel": "k_tile<Poisson,%s,particle targets> (PP+PC)"
                % args.form.upper(), "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None,
                "flop_per_eval": fpe, "evals_per_launch": evals_near,
                "avg_launch_ms": near_ms,
                "valu_slot_frac": (evals_near * SLOTS_PER_EVAL_FP32 / (near_ms / 1e3)
                                   / VALU_SLOTS_PER_S) if args.form == "fp32" else None}
    line = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": r["steps"],
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.form == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "Poisson log kernel, equiangular cubed sphere E=%d (N=%d), "
                               "same set, band-limited n<=32 field (seed 2002), p=%d, theta=%g, "
                               "leaf<=%d, %s form" % (args.E, N, args.p, theta, leaf, args.form),
                   "n": N, "p": args.p, "theta": theta, "leaf": leaf, "form": args.form},
        "rel_l2_err": r["rel"], "max_err": r["max"], "tolerance": 1e-5,
        "meets_tolerance": r["rel"] <= 1e-5,
        "latency_ms": {"p50": float(np.percentile(r["lat"], 50)),
                       "p99": float(np.percentile(r["lat"], 99))},
        "plan_ms": r["plan_ms"],
        "stage_ms": r["stage"],
        "evals": {k: st["evals_" + k] for k in ("pp", "pc", "cp", "cc")},
        "other_form": {f: {"value": float(N) * N / (results[f]["wall"] / results[f]["steps"]),
                           "ms_per_step": 1e3 * results[f]["wall"] / results[f]["steps"],
                           "rel_l2_err": results[f]["rel"], "stage_ms": results[f]["stage"]}
                       for f in results if f != args.form},
        "fp32_over_fp64_speedup": (results["fp64"]["wall"] / results["fp64"]["steps"])
                                  / (results["fp32"]["wall"] / results["fp32"]["steps"]),
        "gpu_direct_rate": direct_rate,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(P, w, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
