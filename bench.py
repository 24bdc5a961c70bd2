"""Benchmark: one CSFMM evaluation per step on one MI355X.

Headline workload (the largest single-GPU configuration): the 1/|x-y|
kernel with 6,291,456 sources on the equiangular cubed sphere (1024 x 1024
cells per face) carrying w = f A for a seeded band-limited field (n <= 64,
coefficient variance (n+1)^-3, seed 4004), and 1,000,000 seeded uniform
random targets (seed 4005); p = 10, theta = 0.6, leaf <= 128.  The headline
line is the plain FP64 form (every step in FP64, the paper's arithmetic);
the FP32 form (FP32 kernel evaluations, FP64 geometry, interpolation and
sums) is reported beside it with its speed-up.  The plan (trees, lists) is
built once before timing; a step is one csfmm_eval: P2M, M2M, PP, PC, CP,
CC, L2L, L2P.  Inputs are resident in HBM before the timed region.

Errors are against the FP64 direct-sum oracle (C, OpenMP) on 4,096 seeded
targets (seed 4006) x all sources; timing that oracle run on the host cores
is the CPU baseline.  Beside the headline: the Poisson workload on
256 x 256 cells per face (N = 393,216) at p = 6, 8, 10 in the FP32 form and
p = 6 in FP64, each against the oracle on its 4,096-target sample.

Prints one JSON line.  Other modes: --copy-calibration times a plain
256 MiB device copy (the reference kernel for scaling HBM byte counters);
--counters DIR folds rocprofv3 counter runs into a record under profiles/.
"""

import argparse
import json
import os
import platform
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "N^2-equiv interactions/s per FMM eval at rel L2 err<=1e-5; p50/p99 latency"
UNIT = "N^2-equiv interactions/s"
TOL = 1e-5
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (published)
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector (published)
# Algorithmic floating point work of one evaluation K(x,y) w of the Poisson
# and 1/|x-y| kernels: |x-y|^2 (3 sub, 3 mul, 2 add) + 1 log or rsqrt + 1
# multiply-add (2) = 11 flops.
FLOP_PER_EVAL = 11
HEADLINE_RECORD = "near_pp_invdist_src6291456_tgt1M_p10_fp64_counters.json"
POISSON_RECORD = "near_pp_poisson_E256_p6_fp32_counters.json"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--form", choices=("fp32", "fp64"), default="fp64",
                    help="form of the headline line (the other one is reported beside it)")
    ap.add_argument("--quick", action="store_true",
                    help="headline form only (no other form, no Poisson lines, no CPU baseline)")
    ap.add_argument("--poisson-cases", default="fp32_p6,fp32_p8,fp32_p10,fp64_p6",
                    help="--poisson-only: which of the Poisson lines to run")
    ap.add_argument("--poisson-only", action="store_true",
                    help="only the Poisson N=393,216 lines (its kernels for profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--counters", metavar="DIR",
                    help="fold the rocprofv3 csv runs under DIR into a profiles/ record")
    ap.add_argument("--record", default=HEADLINE_RECORD, help="record name for --counters")
    ap.add_argument("--serve", action="store_true", help="serving stream instead (2,000 requests)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rho", type=float, nargs="*", default=[0.5, 0.8])
    ap.add_argument("--streams", type=int, default=3, help="serving: compute streams")
    ap.add_argument("--sweep", action="store_true",
                    help="runtime vs error over degree, MAC, leaf size and form (Fig. 7 analogue)")
    ap.add_argument("--sweep-E", type=int, default=330)
    ap.add_argument("--sweep-kernels", type=int, nargs="*", default=[1, 4])
    ap.add_argument("--table2", action="store_true",
                    help="paper Table 2 on the icosahedral grid N=655,362 (error vs MAC, n)")
    ap.add_argument("--table3", action="store_true",
                    help="paper Table 3 on icosahedral grids (runtime vs N, four kernels)")
    ap.add_argument("--table3-kmax", type=int, default=9)
    ap.add_argument("--bve", action="store_true",
                    help="barotropic vorticity equation, Rossby-Haurwitz wave, RK4 (paper §12)")
    ap.add_argument("--bve-k", type=int, default=7)
    ap.add_argument("--bve-e", type=int, default=165,
                    help="cubed-sphere cells per face edge of the remeshed BVE runs")
    ap.add_argument("--configs", action="store_true",
                    help="the other workloads: Poisson E=32, Biot-Savart E=512, 1/|x-y| 6.3M x 1M")
    ap.add_argument("--extras", action="store_true",
                    help="also the per-kernel table and the treecode on the Poisson grid")
    return ap.parse_args()


def say(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def source_sha(name="tile.hip"):
    import hashlib
    return hashlib.sha256(open(os.path.join(ROOT, "paper_2508_13550_amd", "csrc", name),
                               "rb").read()).hexdigest()


def recorded_traffic(name):
    """The committed counter record `name`, or None when the tile kernel's
    source has changed since it was taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
    except (OSError, ValueError):
        return None
    return rec if rec.get("tile_hip_sha256") == source_sha() else None


def host_cpu():
    """Model name of the host CPU (lscpu), for the CPU-baseline record."""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return platform.processor() or platform.machine()


def _norms(x):
    x = np.asarray(x, dtype=np.float64)
    return np.abs(x) if x.ndim == 1 else np.sqrt(np.sum(x * x, axis=1))


def errors(got, ref, area=None):
    """rel L2 (area weights or 1), max err (max |d| / max |ref|) and the
    worst per-target error floored at the sample RMS, against the oracle."""
    d, r = _norms(np.asarray(got) - ref), _norms(ref)
    a = np.ones_like(r) if area is None else area
    rms = float(np.sqrt(np.mean(r * r)))
    return {"rel_l2_err": float(np.sqrt(np.sum(a * d * d) / np.sum(a * r * r))),
            "max_err": float(np.max(d) / np.max(r)),
            "elem_max_err": float(np.max(d / np.maximum(r, rms)))}


def copy_calibration():
    import torch
    n = 256 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))


KERNEL_NAMES = {1: "poisson", 2: "biot_savart", 3: "inv_dist", 4: "biharmonic", 5: "sal"}


def kernel_table(cs, torch, T, W, N, p, theta, leaf, S, steps):
    """Eval time and error of every kernel on the headline geometry (one plan
    per form, kernel chosen per eval), like the paper's Table 3 rows; the
    error is against the GPU FP64 direct sum on the 4,096-target sample."""
    Ts = T[S].contiguous()
    table = {}
    for k, name in KERNEL_NAMES.items():
        ref = cs.direct(Ts, T, W, kernel=k)
        table[name] = {}
        for fp32 in (True, False):
            plan = cs.Plan(T, None, kernel=k, p=p, theta=theta, leaf_size=leaf, fp32=fp32)
            out = plan.eval(W)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                plan.eval(W, out=out)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / steps
            plan.close()
            d = out[S] - ref
            rel = float(torch.sqrt(torch.sum(d * d) / torch.sum(ref * ref)))
            table[name]["fp32" if fp32 else "fp64"] = {"ms": ms, "rel_l2_err": rel}
    return table


def treecode_line(cs, torch, T, W, N, p, theta, leaf, S, ref_s, steps=5):
    """The cubed sphere treecode (Algorithm 1, FP64) on the headline geometry,
    beside the FP64 CSFMM eval on the same plan (the paper compares the two)."""
    plan = cs.Plan(T, None, kernel=cs.POISSON, p=p, theta=theta, leaf_size=leaf)
    res = {}
    for name, fn in (("cstc", plan.eval_treecode), ("csfmm", plan.eval)):
        out = fn(W)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn(W, out=out)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        d = out[S] - ref_s
        res[name] = {"ms": ms, "rel_l2_err": float(torch.sqrt(torch.sum(d * d) /
                                                              torch.sum(ref_s * ref_s)))}
    plan.close()
    res["form"] = "fp64"
    res["csfmm_speedup"] = res["cstc"]["ms"] / res["csfmm"]["ms"]
    return res


SWEEP_TOLS = (1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10, 1e-11, 1e-12)


def sweep_bench(args):
    """Eval time vs approximation error over p = 2:2:14, MAC in {0.5, 0.7, 0.9},
    leaf size in {64, 128, 256, 4p^2} (4p^2 is the paper's N0) and both forms,
    for the Poisson and biharmonic kernels (the paper's Fig. 7 pair), on the
    cubed-sphere grid closest to the paper's N = 655,362 (E = 330: 653,400
    points) with the band-limited field of the headline workload.  Error:
    relative L2 against the GPU FP64 direct sum on 4,096 seeded targets.
    Prints every point, the Pareto front per kernel, and the fastest setting
    per tolerance."""
    import torch
    import paper_2508_13550_amd as cs
    from workloads import make_config, config_subset

    cfg = make_config(2, E=args.sweep_E)
    P, w = cfg["sources"], cfg["weights"]
    N = P.shape[0]
    dev = torch.device("cuda:0")
    T = torch.tensor(P, dtype=torch.float64, device=dev)
    W = torch.tensor(w, dtype=torch.float64, device=dev)
    S = torch.tensor(config_subset(N, 4096, cfg["subset_seed"]), device=dev)
    Ts = T[S].contiguous()
    points = []
    for k in args.sweep_kernels:
        ref = cs.direct(Ts, T, W, kernel=k)
        for theta in (0.5, 0.7, 0.9):
            for p in range(2, 15, 2):
                for leaf in sorted({64, 128, 256, 4 * p * p}):
                    for fp32 in (True, False):
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        plan = cs.Plan(T, None, kernel=k, p=p, theta=theta, leaf_size=leaf,
                                       fp32=fp32)
                        torch.cuda.synchronize()
                        plan_ms = 1e3 * (time.perf_counter() - t0)
                        out = plan.eval(W)
                        plan.eval(W, out=out)
                        torch.cuda.synchronize()
                        reps = 10
                        t0 = time.perf_counter()
                        for _ in range(reps):
                            plan.eval(W, out=out)
                        torch.cuda.synchronize()
                        ms = 1e3 * (time.perf_counter() - t0) / reps
                        plan.close()
                        d = out[S] - ref
                        rel = float(torch.sqrt(torch.sum(d * d) / torch.sum(ref * ref)))
                        points.append({"kernel": KERNEL_NAMES[k], "theta": theta, "p": p,
                                       "leaf": leaf, "form": "fp32" if fp32 else "fp64",
                                       "ms": ms, "rel_l2_err": rel, "plan_ms": plan_ms})
                    print("sweep %s theta %.1f p %d done" % (KERNEL_NAMES[k], theta, p),
                          file=sys.stderr, flush=True)
    fronts, best = {}, {}
    for k in args.sweep_kernels:
        name = KERNEL_NAMES[k]
        pts = sorted((q for q in points if q["kernel"] == name), key=lambda q: q["ms"])
        front, lo = [], float("inf")
        for q in pts:
            if q["rel_l2_err"] < lo:
                front.append(q)
                lo = q["rel_l2_err"]
        fronts[name] = front
        best[name] = {}
        for tol in SWEEP_TOLS:
            ok = [q for q in pts if q["rel_l2_err"] <= tol]
            best[name]["%g" % tol] = ok[0] if ok else None
    line = {"metric": "eval time vs relative L2 error (p, MAC, leaf, form sweep)",
            "unit": "ms", "n_gpus": 1, "data": "synthetic",
            "config": {"workload": "equiangular cubed sphere %dx%d cells per face (N=%d), "
                                   "band-limited n<=32 field (seed 2002)"
                                   % (args.sweep_E, args.sweep_E, N), "n": N},
            "points": points, "pareto": fronts, "fastest_within_tol": best}
    print(json.dumps(line), flush=True)


def _golden_rows(name):
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


def table2_bench(args):
    """The paper's Table 2 at its own setting: icosahedral grid N = 655,362,
    N0 = 4 n^2, fields Y00, Y43, Y85, MAC 0.9/0.7/0.5, n = 2:2:14, FP64.
    E(phi_FS, phi_DS) = ||phi_FS - phi_DS|| / ||phi_EX|| with area weights,
    phi_EX = f/(n(n+1)) (Y00: its exact constant), phi_DS the GPU FP64 direct
    sum at every point."""
    import math
    import torch
    import paper_2508_13550_amd as cs
    from workloads import icosahedral_grid, real_sph_harm_all

    P, A = icosahedral_grid(8)
    N = P.shape[0]
    dev = torch.device("cuda:0")
    T = torch.tensor(P, dtype=torch.float64, device=dev)
    Y = real_sph_harm_all(P, 8)
    y00 = 1.0 / (2.0 * math.sqrt(math.pi))
    fields = {"Y00": (np.full(N, y00), (1.0 - math.log(2.0)) / (2.0 * math.sqrt(math.pi))),
              "Y43": (Y[:, 4 * 4 + 4 + 3], 1.0 / 20.0),
              "Y85": (Y[:, 8 * 8 + 8 + 5], 1.0 / 72.0)}
    paper = {(r[0], float(r[1])): [float(v) for v in r[2:]] for r in _golden_rows("table2_full.txt")}
    data = {}
    for name, (f, lam) in fields.items():
        W = torch.tensor(f * A, dtype=torch.float64, device=dev)
        ds = cs.direct(T, T, W, kernel=cs.POISSON).cpu().numpy()
        ex = (np.full(N, lam) if name == "Y00" else lam * f)
        nex = math.sqrt(np.sum(ex * ex * A))
        data[name] = (W, ds, nex, math.sqrt(np.sum((ds - ex) ** 2 * A)) / nex)
        print("table2 direct %s done" % name, file=sys.stderr, flush=True)
    rows = []
    for theta in (0.9, 0.7, 0.5):
        for n in range(2, 15, 2):
            plan = cs.Plan(T, None, kernel=cs.POISSON, p=n, theta=theta, leaf_size=4 * n * n)
            for name in fields:
                W, ds, nex, _ = data[name]
                out = plan.eval(W)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan.eval(W, out=out)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0)
                fs = out.cpu().numpy()
                e = math.sqrt(np.sum((fs - ds) ** 2 * A)) / nex
                pe = paper[(name, theta)][n // 2 - 1]
                rows.append({"field": name, "theta": theta, "n": n, "leaf": 4 * n * n,
                             "E": e, "paper_E": pe, "ratio": e / pe, "eval_ms": ms})
            plan.close()
            print("table2 theta %.1f n %d done" % (theta, n), file=sys.stderr, flush=True)
    line = {"metric": "paper Table 2: E(phi_FS, phi_DS) vs MAC and degree (FP64)",
            "n_gpus": 1, "data": "synthetic",
            "config": {"workload": "icosahedral grid k=8 (N=%d), N0=4n^2, Poisson kernel" % N},
            "discretization_error": {k: v[3] for k, v in data.items()}, "rows": rows}
    print(json.dumps(line), flush=True)


def table3_bench(args):
    """The paper's Table 3 on one MI355X: icosahedral grids N = 10*4^k + 2,
    k = 4..9, MAC 0.7, n = 6, N0 = 4n^2 = 144, four kernels.  CSFMM: mean of
    3 evals (FP64 and FP32 form); direct: the GPU direct sum timed on 8,192
    targets against all N sources and scaled by N/8,192 (its cost is linear in
    the number of targets)."""
    import torch
    import paper_2508_13550_amd as cs
    from workloads import icosahedral_grid, real_y43

    kernels = {"laplace": cs.POISSON, "biharmonic": cs.BIHARMONIC,
               "biot_savart": cs.BIOT_SAVART, "sal": cs.SAL}
    paper = {(r[0], r[1]): [float(v) for v in r[2:]] for r in _golden_rows("table3_runtimes.txt")}
    dev = torch.device("cuda:0")
    rows = []
    for k in range(4, args.table3_kmax + 1):
        P, A = icosahedral_grid(k)
        N = P.shape[0]
        T = torch.tensor(P, dtype=torch.float64, device=dev)
        W = torch.tensor(real_y43(P) * A, dtype=torch.float64, device=dev)
        nsub = min(N, 8192)
        Ts = T[:nsub].contiguous()
        for name, kid in kernels.items():
            row = {"N": N, "kernel": name}
            for fp32 in (False, True):
                plan = cs.Plan(T, None, kernel=kid, p=6, theta=0.7, leaf_size=144, fp32=fp32)
                out = plan.eval(W)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(3):
                    plan.eval(W, out=out)
                torch.cuda.synchronize()
                row["csfmm_%s_s" % ("fp32" if fp32 else "fp64")] = (time.perf_counter() - t0) / 3
                plan.close()
                cs.direct(Ts, T, W, kernel=kid, fp32=fp32)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                cs.direct(Ts, T, W, kernel=kid, fp32=fp32)
                torch.cuda.synchronize()
                row["direct_%s_s" % ("fp32" if fp32 else "fp64")] = \
                    (time.perf_counter() - t0) * N / nsub
            col = k - 4
            row["paper_direct_s"] = paper[("direct", name)][col]
            row["paper_csfmm_s"] = paper[("csfmm", name)][col]
            row["speedup_vs_paper_csfmm_fp64"] = row["paper_csfmm_s"] / row["csfmm_fp64_s"]
            row["speedup_vs_paper_csfmm_fp32"] = row["paper_csfmm_s"] / row["csfmm_fp32_s"]
            rows.append(row)
            print("table3 N %d %s done" % (N, name), file=sys.stderr, flush=True)
    line = {"metric": "paper Table 3: runtime (s) vs N, direct and CSFMM, four kernels",
            "n_gpus": 1, "data": "synthetic",
            "config": {"workload": "icosahedral grids k=4..%d, MAC 0.7, n=6, N0=144, "
                                   "f = Re Y_4^3" % args.table3_kmax},
            "rows": rows}
    print(json.dumps(line), flush=True)


def bve_bench(args):
    """The paper's §12 Rossby-Haurwitz run: icosahedral particles (k = 7:
    N = 163,842), RK4 with dt = 0.01 day to t = 1 day, velocity by CSFMM
    (MAC 0.7, n = 6, leaf 4n^2; FP64 and the FP32 form) and by the FP64 direct
    sum (timed over the first 10 steps, error after 100); every stage rebuilds
    the plan.  Reports time per step and E_zeta at 1 day (eq. bveerr).  The
    same run on the cubed-sphere grid remeshed after every step (§12) times
    the step with its remesh, and the remesh alone over the first 10 steps."""
    import torch
    import paper_2508_13550_amd as cs
    from workloads import icosahedral_grid, rh_vorticity

    def vorticity_error(x, z):   # eq. (bveerr) against the stationary wave
        z0 = rh_vorticity(x)
        return float(np.sqrt(np.sum((z - z0) ** 2 * A) / np.sum(z0 ** 2 * A)))

    P, A = icosahedral_grid(args.bve_k)
    N = P.shape[0]
    a = torch.tensor(A, dtype=torch.float64, device="cuda")
    runs = {}
    for name, kw in (("csfmm_fp64", dict(fp32=False, use_direct=False)),
                     ("csfmm_fp32", dict(fp32=True, use_direct=False)),
                     ("direct_fp64", dict(fp32=False, use_direct=True))):
        x = torch.tensor(P, dtype=torch.float64, device="cuda")
        z = torch.tensor(rh_vorticity(P), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t10 = None
        for step in range(100):
            cs.bve_rk4_step(x, z, a, 0.01, p=6, theta=0.7, leaf_size=144, **kw)
            if step == 9:
                torch.cuda.synchronize()
                t10 = time.perf_counter() - t0
            if (step + 1) % 20 == 0:
                print("bve %s step %d" % (name, step + 1), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        e = vorticity_error(x.cpu().numpy(), z.cpu().numpy())
        runs[name] = {"s_per_step": total / 100, "s_per_step_first10": t10 / 10,
                      "E_zeta_1day": e}
    # remeshed after every step (csfmm_bve_remesh) on the cubed-sphere grid
    from workloads import cubed_sphere_grid
    E = args.bve_e
    Pc, Ac = cubed_sphere_grid(E)
    Nc = Pc.shape[0]
    ac = torch.tensor(Ac, dtype=torch.float64, device="cuda")
    g = torch.tensor(Pc, dtype=torch.float64, device="cuda")
    for name, kw in (("csfmm_fp64_remeshed", dict(fp32=False, use_direct=False)),
                     ("direct_fp64_remeshed", dict(fp32=False, use_direct=True))):
        x = g.clone()
        z = torch.tensor(rh_vorticity(Pc), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_rm = 0.0
        for step in range(100):
            cs.bve_rk4_step(x, z, ac, 0.01, p=6, theta=0.7, leaf_size=144, **kw)
            if step < 10:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
            cs.bve_remesh(g, E, x, z)
            if step < 10:
                torch.cuda.synchronize()
                t_rm += time.perf_counter() - t1
            if (step + 1) % 20 == 0:
                print("bve %s step %d" % (name, step + 1), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        zc = z.cpu().numpy()
        z0 = rh_vorticity(Pc)
        e = float(np.sqrt(np.sum((zc - z0) ** 2 * Ac) / np.sum(z0 ** 2 * Ac)))
        runs[name] = {"s_per_step": total / 100, "remesh_s_per_step_first10": t_rm / 10,
                      "E_zeta_1day": e}
    line = {"metric": "BVE Rossby-Haurwitz wave: time per RK4 step and E_zeta at 1 day",
            "n_gpus": 1, "data": "synthetic",
            "config": {"workload": "icosahedral k=%d (N=%d), dt=0.01 day, 100 steps, "
                                   "MAC 0.7, n=6, leaf 144; remeshed runs: cubed-sphere "
                                   "E=%d (N=%d), remeshed after every step"
                                   % (args.bve_k, N, E, Nc)},
            "runs": runs,
            "csfmm_speedup_over_direct": runs["direct_fp64"]["s_per_step"] /
            runs["csfmm_fp64"]["s_per_step"],
            "csfmm_speedup_over_direct_remeshed": runs["direct_fp64_remeshed"]["s_per_step"] /
            runs["csfmm_fp64_remeshed"]["s_per_step"]}
    print(json.dumps(line), flush=True)


def configs_bench(args):
    """Throughput of the workloads beside the headline one, each in the form
    and parameters it is specified with: Poisson E=32 (FP64, p=8, theta 0.7,
    leaf 64; 100 evals), Biot-Savart E=512 (FP32 form, p=8, theta 0.6, leaf 128;
    30 evals), 1/|x-y| with 6,291,456 sources and 1,000,000 random targets
    (FP32 form, p=10, theta 0.6, leaf 128; 10 evals).  Plan time is reported
    apart; the error is relative L2 on 4,096 seeded targets (all 6,144 for the
    small one) against the GPU FP64 direct sum."""
    import torch
    import paper_2508_13550_amd as cs
    from workloads import make_config, config_subset

    rows = []
    for cid, fp32, reps in ((1, False, 100), (3, True, 30), (4, True, 10)):
        c = make_config(cid)
        print("configs: inputs of workload %d ready" % cid, file=sys.stderr, flush=True)
        S = c["sources"]
        T = S if c["targets"] is None else c["targets"]
        dev = torch.device("cuda:0")
        Sd = torch.tensor(S, dtype=torch.float64, device=dev)
        Td = Sd if c["targets"] is None else torch.tensor(T, dtype=torch.float64, device=dev)
        W = torch.tensor(c["weights"], dtype=torch.float64, device=dev)
        nt, ns = T.shape[0], S.shape[0]
        samp = np.arange(nt) if cid == 1 else config_subset(nt, 4096, c["subset_seed"])
        sd = torch.tensor(samp, device=dev)
        ref = cs.direct(Td[sd].contiguous(), Sd, W, kernel=c["kernel"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = cs.Plan(Td, None if c["targets"] is None else Sd, kernel=c["kernel"], p=c["p"],
                       theta=c["theta"], leaf_size=c["leaf"], fp32=fp32)
        torch.cuda.synchronize()
        plan_ms = 1e3 * (time.perf_counter() - t0)
        out = plan.eval(W)
        for _ in range(3):
            plan.eval(W, out=out)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in ev:
            a.record()
            plan.eval(W, out=out)
            b.record()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        lat = np.array([a.elapsed_time(b) for a, b in ev])
        st = plan.stats()
        plan.close()
        d = (out[sd] - ref).reshape(len(samp), -1)
        r = ref.reshape(len(samp), -1)
        if cid == 1 or cid == 3:
            a_w = torch.tensor(c["areas"][samp], dtype=torch.float64, device=dev)[:, None]
        else:
            a_w = torch.ones((len(samp), 1), dtype=torch.float64, device=dev)
        rel = float(torch.sqrt(torch.sum(a_w * d * d) / torch.sum(a_w * r * r)))
        rows.append({"workload": c["name"], "n_targets": nt, "n_sources": ns,
                     "form": "fp32" if fp32 else "fp64", "p": c["p"], "theta": c["theta"],
                     "leaf": c["leaf"], "evals_timed": reps, "ms_per_eval": ms,
                     "latency_ms": {"p50": float(np.percentile(lat, 50)),
                                    "p99": float(np.percentile(lat, 99))},
                     "n2eq_per_s": float(nt) * ns / (ms / 1e3), "plan_ms": plan_ms,
                     "rel_l2_err": rel, "evals": {k: st["evals_" + k] for k in ("pp", "pc", "cp", "cc")},
                     "device_bytes": st["device_bytes"]})
        print("configs: workload %d done" % cid, file=sys.stderr, flush=True)
        del Sd, Td, W, out, ref
        torch.cuda.empty_cache()
    line = {"metric": "N^2-equiv interactions/s per FMM eval, other workloads", "n_gpus": 1,
            "data": "synthetic", "rows": rows}
    print(json.dumps(line), flush=True)


def serve_bench(args):
    """Serving stream: requests of mixed resolution, kernel and degree arriving
    as a Poisson process at rho x capacity; continuous batching on one GPU."""
    import torch
    import paper_2508_13550_amd as cs
    from paper_2508_13550_amd.serve import Server, Request, latency_stats, plan_key
    from workloads import cubed_sphere_grid, real_sph_harm_all, config_subset
    from workloads.serving import request_mix, poisson_arrivals, E_CHOICES

    theta, leaf = 0.6, 128
    n = args.requests
    mix = request_mix(n)
    dev = torch.device("cuda:0")
    grids = {}
    for E in E_CHOICES:
        P, A = cubed_sphere_grid(E)
        Y = real_sph_harm_all(P, 8)
        grids[E] = (torch.tensor(P, device=dev), torch.tensor(Y, device=dev),
                    torch.tensor(A, device=dev))
    W = [(grids[E][1] @ torch.tensor(c, device=dev)) * grids[E][2] for E, k, p, c in mix]
    nn = [6 * E * E for E, k, p, c in mix]
    # solo service time per class with resident plans (capacity = 1 / mean service time)
    plans = {}
    solo = {}
    for E, k, p, c in mix:
        if (E, k, p) in solo:
            continue
        if (E, p) not in plans:
            plans[(E, p)] = cs.Plan(grids[E][0], None, kernel=k, p=p, theta=theta,
                                    leaf_size=leaf, fp32=True)
        pl = plans[(E, p)]
        w = W[[i for i, m in enumerate(mix) if m[:3] == (E, k, p)][0]]
        pl.eval(w, kernel=k)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            pl.eval(w, kernel=k)
        b.record()
        torch.cuda.synchronize()
        solo[(E, k, p)] = a.elapsed_time(b) / 5 / 1e3
    for pl in plans.values():
        pl.close()
    mean_service = float(np.mean([solo[m[:3]] for m in mix]))
    capacity = 1.0 / mean_service
    free, total = torch.cuda.mem_get_info()
    budget = int(0.9 * free)
    results = []
    samples = config_subset(n, 50, 5007)
    for rho in args.rho:
        srv = Server(budget_bytes=budget, theta=theta, leaf=leaf, fp32=True, max_batch=32,
                     n_streams=args.streams)
        # warm the plan cache: one request per (E, p)
        warm, seen = [], set()
        for i, (E, k, p, c) in enumerate(mix):
            if (E, p) not in seen:
                seen.add((E, p))
                warm.append(Request(id=-1 - len(warm), geometry=("grid", E), targets=grids[E][0],
                                    sources=None, kernel=k, p=p, weights=W[i]))
        srv.run(warm)
        srv.done.clear()
        srv.batch_sizes.clear()
        arr = poisson_arrivals(n, rho * capacity, seed=5005)
        reqs = [Request(id=i, geometry=("grid", E), targets=grids[E][0], sources=None,
                        kernel=k, p=p, weights=W[i], t_arrival=float(arr[i]))
                for i, (E, k, p, c) in enumerate(mix)]
        t0 = time.perf_counter()
        done = srv.run(reqs)
        makespan = time.perf_counter() - t0
        st = srv.sched.stats()
        lat = latency_stats(done)
        by_e = {}
        for E in E_CHOICES:
            sel = [r for r in done if r.geometry[1] == E]
            if sel:
                by_e[str(E)] = dict(latency_stats(sel),
                                    solo_ms=float(np.mean([solo[(E, r.kernel, r.p)] for r in sel])) * 1e3)
        # accuracy and alone-vs-mix identity on 50 sampled requests
        by_id = {r.id: r for r in done}
        worst, same = 0.0, True
        for i in samples:
            r = by_id[int(i)]
            E = mix[i][0]
            T = grids[E][0]
            pl = srv.plans[plan_key(("grid", E), r.p, theta, leaf, True)]
            alone = pl.eval(r.weights, kernel=r.kernel)
            same = same and bool(torch.equal(alone, r.out))
            S = torch.tensor(config_subset(T.shape[0], 1024, 5008), device=dev)
            ref = cs.direct(T[S].contiguous(), T, r.weights, kernel=r.kernel)
            got = r.out[S]
            err = float(torch.sqrt(torch.sum((got - ref) ** 2) / torch.sum(ref ** 2)))
            worst = max(worst, err)
        n2 = float(sum(x * x for x in nn))
        results.append({"rho": rho, "arrival_rate_per_s": rho * capacity,
                        "latency_ms": lat, "makespan_s": makespan,
                        "throughput_req_per_s": len(done) / makespan,
                        "throughput_n2eq_per_s": n2 / makespan,
                        "mean_batch": float(np.mean(srv.batch_sizes)),
                        "max_batch": int(max(srv.batch_sizes)),
                        "max_concurrent_batches": srv.max_concurrent,
                        "latency_by_E": by_e, "host_s": srv.host_s,
                        "p99_over_mean_service": lat["p99_ms"] / (mean_service * 1e3),
                        "sched": st, "sample_max_rel_l2": worst, "alone_equals_mix": same})
        srv.close()
    line = {"metric": "serving: p50/p99 latency and throughput of a CSFMM request stream",
            "n_requests": n, "streams": args.streams, "capacity_req_per_s": capacity, "mean_solo_service_ms":
            mean_service * 1e3, "budget_bytes": budget, "theta": theta, "leaf": leaf,
            "form": "fp32", "n_gpus": 1, "data": "synthetic",
            "config": {"workload": "2,000 requests, E in {16..512} (N 1,536..1,572,864), "
                                   "kernel in {Poisson, Biot-Savart, 1/|x-y|}, p in {6, 8}, "
                                   "Poisson arrivals (seed 5005)"},
            "runs": results}
    print(json.dumps(line), flush=True)


def measure(cs, torch, Td, Sd, W, kernel, p, theta, leaf, fp32, steps, warmup, samp):
    """Plan once, then: warm-up evals; `steps` timed evals with HIP events
    around the PP launch (side stream) and the PC + far-field launch (eval
    stream) and nothing else recorded; a latency pass with events around every
    eval; a stage-breakdown pass.  Returns times, stats and the outputs at the
    sampled targets (host)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = cs.Plan(Td, Sd, kernel=kernel, p=p, theta=theta, leaf_size=leaf, fp32=fp32)
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t0)
    out = plan.eval(W)
    for _ in range(warmup):
        plan.eval(W, out=out)
    torch.cuda.synchronize()
    plan.timing(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.eval(W, out=out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_t, st_t = plan.timing_read()
    plan.timing(False)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(min(steps, 100))]
    for a, b in ev:
        a.record()
        plan.eval(W, out=out)
        b.record()
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    plan.timing(1)
    for _ in range(max(5, min(50, steps // 4))):
        plan.eval(W, out=out)
    n, stage = plan.timing_read()
    plan.timing(False)
    stage = {k: v / max(n, 1) for k, v in stage.items()}
    stage["near_pp_timed_region"] = st_t["near_pp"] / max(n_t, 1)
    stage["pc_far_timed_region"] = st_t["pc_far"] / max(n_t, 1)
    stage["interaction_span_timed_region"] = st_t["interaction_span"] / max(n_t, 1)
    st = plan.stats()
    plan.close()
    got = out[torch.as_tensor(samp, device=out.device)].cpu().numpy()
    ms = 1e3 * wall / steps
    del out
    torch.cuda.empty_cache()
    return dict(p=p, form="fp32" if fp32 else "fp64", plan_ms=plan_ms, ms=ms, steps=steps,
                lat=lat, stage=stage, stats=st, got=got)


def pp_grid(st):
    """Work-items of the PP launch: four target leaves per block on the
    one-wave-per-leaf path, else one leaf per block; 256 threads a block."""
    nl = st["n_leaves_t"]
    return 256 * ((nl + 3) // 4 if st["near_wave"] else nl)


def roofline_of(r, fp32, record_name, kernel_desc):
    """Roofline of the interaction launches, the dominant kernel: the PP
    launch (side stream) and the PC + far-field launch (eval stream) run
    concurrently, so their evaluations are taken together over the span
    they occupy (the library's HIP events: PP start to the eval stream's join
    with it, in the timed region); each launch's own rate over its own
    event-timed duration is reported beside it."""
    st, stage = r["stats"], r["stage"]
    peak = PEAK_FP32_TFLOPS if fp32 else PEAK_FP64_TFLOPS
    ev_far = st["evals_pc"] + st["evals_cp"] + st["evals_cc"]
    pp_ms, far_ms = stage["near_pp_timed_region"], stage["pc_far_timed_region"]
    span = stage.get("interaction_span_timed_region", 0.0)
    span = max(span, pp_ms, far_ms)  # the span holds both launches
    parts = {
        "pp": {"kernel": kernel_desc + ": PP near-field launch", "evals": st["evals_pp"],
               "ms": pp_ms},
        "pc_far": {"kernel": kernel_desc + ": PC near field + CP/CC far field launch",
                   "evals": ev_far, "ms": far_ms}}
    for q in parts.values():
        q["achieved"] = q["evals"] * FLOP_PER_EVAL / (q["ms"] / 1e3) / 1e12 if q["ms"] > 0 else 0.0
        q["frac"] = q["achieved"] / peak
    evals = st["evals_pp"] + ev_far
    achieved = evals * FLOP_PER_EVAL / (span / 1e3) / 1e12 if span > 0 else 0.0
    rec = recorded_traffic(record_name)
    traffic = None
    if rec:
        # the record is of this workload when its PP launch has this grid; the
        # PC + far launch is its other k_tile dispatch
        disp = rec.get("dispatches", [])
        g = pp_grid(st)
        pp_rows = [x for x in disp if x["grid_size"] == g and x["pp"]]
        far_rows = [x for x in disp if not x["pp"] and re.search(r"::k_tile<", x["kernel"])]
        if pp_rows and far_rows:
            traffic = sum(x["traffic_bytes"] for x in pp_rows + far_rows)
    return {"bound": "alu",
            "kernel": kernel_desc + ": the PP launch and the PC + far launch, concurrent",
            "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": traffic, "flop_per_eval": FLOP_PER_EVAL, "evals_per_step": evals,
            "span_ms": span, "launches": parts,
            "traffic_record": record_name if traffic is not None else None}


def cpu_baseline_of(t_oracle, n_samp, n_src, what):
    from oracle import oracle_threads
    return {"value": n_samp * n_src / t_oracle, "unit": UNIT, "cores": oracle_threads(),
            "kind": "oracle",
            "sample": "FP64 direct-sum oracle (C, OpenMP) on %s: %d seeded targets x all %d "
                      "sources in %.1f s; the direct method's pairs/s is its N^2-equiv rate"
                      % (what, n_samp, n_src, t_oracle),
            "host_cpu": host_cpu()}


def poisson_lines(cs, torch, args):
    """The Poisson workload N = 393,216 (theta 0.7, leaf 128) at p = 6, 8, 10
    in the FP32 form and p = 6 in FP64, against the oracle on its sample."""
    from oracle import direct as odirect
    from workloads import make_config, config_subset
    c = make_config(2)
    P, w, A = c["sources"], c["weights"], c["areas"]
    N = P.shape[0]
    S = config_subset(N, 4096, c["subset_seed"])
    say("poisson: oracle on 4,096 targets x %d sources" % N)
    ref = odirect(1, P[S], P, w)
    dev = torch.device("cuda:0")
    T = torch.tensor(P, dtype=torch.float64, device=dev)
    W = torch.tensor(w, dtype=torch.float64, device=dev)
    steps = max(5, args.steps // 4)
    res = {}
    cases = [(fp32, p) for fp32, p in ((True, 6), (True, 8), (True, 10), (False, 6))
             if not args.poisson_only or
             "%s_p%d" % ("fp32" if fp32 else "fp64", p) in args.poisson_cases.split(",")]
    for fp32, p in cases:
        r = measure(cs, torch, T, None, W, 1, p, c["theta"], c["leaf"], fp32, steps,
                    max(2, args.warmup // 2), S)
        e = errors(r["got"], ref, A[S])
        key = "%s_p%d" % (r["form"], p)
        res[key] = {"ms_per_step": r["ms"], "value": float(N) * N / (r["ms"] / 1e3),
                    "latency_ms": {"p50": float(np.percentile(r["lat"], 50)),
                                   "p99": float(np.percentile(r["lat"], 99))},
                    "plan_ms": r["plan_ms"], "stage_ms": r["stage"],
                    "evals": {k: r["stats"]["evals_" + k] for k in ("pp", "pc", "cp", "cc")},
                    "pp_close": r["stats"]["pp_close"], **e}
        if fp32 and p == 6:
            res[key]["roofline"] = roofline_of(r, True, POISSON_RECORD,
                                               "Poisson FP32 (PP: k_tile_wave + k_sym_merge; "
                                               "PC + far: k_tile)")
        say("poisson %s done: %.4f ms, rel L2 %.2e" % (key, r["ms"], e["rel_l2_err"]))
    if "fp64_p6" in res and "fp32_p6" in res:
        res["fp32_over_fp64_speedup_p6"] = (res["fp64_p6"]["ms_per_step"] /
                                            res["fp32_p6"]["ms_per_step"])
    res["workload"] = ("Poisson log kernel, equiangular cubed sphere 256x256 cells per face "
                       "(N=%d), same set, band-limited n<=32 field (seed 2002), theta=%g, "
                       "leaf<=%d" % (N, c["theta"], c["leaf"]))
    res["error_reference"] = "oracle direct sum on 4,096 seeded targets (seed 2003)"
    extras = None
    if args.extras:
        Sd = torch.tensor(S, device=dev)
        ref_s = torch.tensor(ref, device=dev)
        extras = {"kernels": kernel_table(cs, torch, T, W, N, 6, c["theta"], c["leaf"], Sd, 10),
                  "treecode": treecode_line(cs, torch, T, W, N, 6, c["theta"], c["leaf"], Sd,
                                            ref_s)}
    return res, extras


def fold_counters(args):
    """Fold rocprofv3 --pmc csv runs into profiles/<record>: DIR holds the runs
    FETCH_SIZE, WRITE_SIZE (the benchmark), FETCH_SIZE_copy, WRITE_SIZE_copy
    (--copy-calibration) and optionally SQ; every csv *counter_collection*
    below each is read.  Per dispatch: counters summed over their rows; per
    (kernel, grid size): the mean over its dispatches."""
    import csv
    import glob

    def load(sub):
        rows = {}
        for f in glob.glob(os.path.join(args.counters, sub, "**", "*counter_collection*.csv"),
                           recursive=True):
            for r in csv.DictReader(open(f)):
                key = (r["Kernel_Name"], int(r["Grid_Size"]))
                d = rows.setdefault(key, {})
                dd = d.setdefault(r["Dispatch_Id"], {})
                dd[r["Counter_Name"]] = dd.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        out = {}
        for key, d in rows.items():
            names = set(n for dd in d.values() for n in dd)
            out[key] = {"dispatches": len(d),
                        **{n: float(np.mean([dd.get(n, 0.0) for dd in d.values()])) for n in names}}
        return out

    fetch, write = load("FETCH_SIZE"), load("WRITE_SIZE")
    cf, cw = load("FETCH_SIZE_copy"), load("WRITE_SIZE_copy")
    sq = load("SQ")
    for k, v in load("SQ2").items():
        sq.setdefault(k, {}).update({n: x for n, x in v.items() if n != "dispatches"})
    ck = [k for k in cf if "copyBuffer" in k[0]]
    copy_bytes = 256 * 1024 * 1024
    ffac = copy_bytes / (cf[ck[0]]["FETCH_SIZE"] * 1024.0)
    wfac = copy_bytes / (cw[[k for k in cw if "copyBuffer" in k[0]][0]]["WRITE_SIZE"] * 1024.0)
    disp = []
    for key in sorted(fetch, key=lambda k: -fetch[k]["FETCH_SIZE"]):
        name, grid = key
        if not re.search(r"::(k_tile|k_sym_merge)", name):
            continue
        fk, wk = fetch[key]["FETCH_SIZE"], write.get(key, {}).get("WRITE_SIZE", float("nan"))
        disp.append({"kernel": name, "grid_size": grid, "dispatches": fetch[key]["dispatches"],
                     "fetch_size_kib": fk, "write_size_kib": wk,
                     "traffic_bytes": fk * 1024.0 * ffac + wk * 1024.0 * wfac,
                     "sq": {k: v for k, v in sq.get(key, {}).items() if k.startswith("SQ_")},
                     "pp": False})
    # the PP launch: k_tile_wave and k_sym_merge always, and the k_tile
    # instance for PP launches (its last template argument true)
    for x in disp:
        x["pp"] = (not re.search(r"::k_tile<", x["kernel"]) or
                   re.search(r"::k_tile<\d+, (true|false), true>", x["kernel"]) is not None)
    rec = {"record": args.record, "tile_hip_sha256": source_sha(),
           "copy_calibration": {"bytes": copy_bytes, "fetch_factor": ffac, "write_factor": wfac},
           "dispatches": disp}
    path = os.path.join(ROOT, "profiles", args.record)
    json.dump(rec, open(path, "w"), indent=1)
    print(json.dumps(rec))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1): the library runs on one GPU and has "
              "no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.counters:
        fold_counters(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    for flag, fn in (("serve", serve_bench), ("sweep", sweep_bench), ("table2", table2_bench),
                     ("table3", table3_bench), ("bve", bve_bench), ("configs", configs_bench)):
        if getattr(args, flag):
            fn(args)
            return
    import torch
    import paper_2508_13550_amd as cs
    cs.load_library()
    if args.poisson_only:
        res, extras = poisson_lines(cs, torch, args)
        print(json.dumps({"metric": METRIC, "unit": UNIT, "n_gpus": 1, "poisson_E256": res,
                          "extras": extras}), flush=True)
        return
    from oracle import direct as odirect
    from workloads import make_config, config_subset

    say("headline inputs: 6,291,456 sources (E=1024), 1,000,000 random targets")
    c = make_config(4)
    Y, w, X = c["sources"], c["weights"], c["targets"]
    nt, ns = X.shape[0], Y.shape[0]
    samp = config_subset(nt, 4096, c["subset_seed"])
    say("oracle direct sum on 4,096 targets x %d sources" % ns)
    t0 = time.perf_counter()
    ref = odirect(3, X[samp], Y, w)
    t_oracle = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    Xd = torch.tensor(X, dtype=torch.float64, device=dev)
    Yd = torch.tensor(Y, dtype=torch.float64, device=dev)
    W = torch.tensor(w, dtype=torch.float64, device=dev)
    fp32 = args.form == "fp32"
    kw = dict(kernel=3, p=c["p"], theta=c["theta"], leaf=c["leaf"])
    say("headline form %s: plan + %d warm-up + %d timed evals" % (args.form, args.warmup, args.steps))
    head = measure(cs, torch, Xd, Yd, W, kw["kernel"], kw["p"], kw["theta"], kw["leaf"], fp32,
                   args.steps, args.warmup, samp)
    eh = errors(head["got"], ref)
    say("headline done: %.3f ms per eval, rel L2 %.2e" % (head["ms"], eh["rel_l2_err"]))
    st = head["stats"]
    workload = ("1/|x-y| kernel, 6,291,456 sources on the equiangular cubed sphere 1024x1024 "
                "cells per face with a band-limited n<=64 field (seed 4004) x 1,000,000 uniform "
                "random targets (seed 4005), p=%d, theta=%g, leaf<=%d, %s form"
                % (kw["p"], kw["theta"], kw["leaf"], args.form))
    line = {
        "metric": METRIC, "value": float(nt) * ns / (head["ms"] / 1e3), "unit": UNIT,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64", "data": "synthetic",
        "config": {"workload": workload, "n_targets": nt, "n_sources": ns, "kernel": "inv_dist",
                   "p": kw["p"], "theta": kw["theta"], "leaf": kw["leaf"], "form": args.form},
        **eh, "tolerance": TOL, "meets_tolerance": eh["rel_l2_err"] <= TOL,
        "error_reference": "FP64 direct-sum oracle (C) on 4,096 seeded targets (seed 4006) x "
                           "all sources",
        "latency_ms": {"p50": float(np.percentile(head["lat"], 50)),
                       "p99": float(np.percentile(head["lat"], 99))},
        "plan_ms": head["plan_ms"], "stage_ms": head["stage"],
        "evals": {k: st["evals_" + k] for k in ("pp", "pc", "cp", "cc")},
        "pp_close": st["pp_close"], "device_bytes": st["device_bytes"],
        "roofline": roofline_of(head, fp32, HEADLINE_RECORD,
                                "k_tile<InvDist,%s>" % ("FP32" if fp32 else "FP64")),
    }
    if not args.quick:
        say("other form")
        other = measure(cs, torch, Xd, Yd, W, kw["kernel"], kw["p"], kw["theta"], kw["leaf"],
                        not fp32, max(5, args.steps // 4), max(2, args.warmup // 2), samp)
        eo = errors(other["got"], ref)
        line["other_form"] = {"form": other["form"], "value": float(nt) * ns / (other["ms"] / 1e3),
                              "ms_per_step": other["ms"], "plan_ms": other["plan_ms"],
                              "stage_ms": other["stage"], "pp_close": other["stats"]["pp_close"],
                              "latency_ms": {"p50": float(np.percentile(other["lat"], 50)),
                                             "p99": float(np.percentile(other["lat"], 99))},
                              **eo}
        f32, f64 = (head, other) if fp32 else (other, head)
        line["fp32_over_fp64_speedup"] = f64["ms"] / f32["ms"]
        # same-device direct sum on the sample (the FMM's speed-up on one MI355X)
        Xs = Xd[torch.as_tensor(samp, device=dev)].contiguous()
        rates = {}
        for form in ("fp64", "fp32"):
            cs.direct(Xs, Yd, W, kernel=3, fp32=(form == "fp32"))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cs.direct(Xs, Yd, W, kernel=3, fp32=(form == "fp32"))
            torch.cuda.synchronize()
            rates[form] = len(samp) * ns / (time.perf_counter() - t0)
        line["gpu_direct_rate"] = rates
        line["fmm_over_gpu_direct_fp64"] = line["value"] / rates["fp64"] if not fp32 else None
        del Xs
        del Xd, Yd, W
        torch.cuda.empty_cache()
        say("poisson lines")
        line["poisson_E256"], extras = poisson_lines(cs, torch, args)
        if extras:
            line["extras"] = extras
    if not args.no_cpu_baseline and not args.quick:
        line["cpu_baseline"] = cpu_baseline_of(t_oracle, len(samp), ns,
                                               "the headline workload (1/|x-y|)")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
