#!/usr/bin/env python3
"""Benchmark of the CP-ALS relaxation sweep on one MI355X.

Workload: dense 256 x 256 x 256 tensor, rank R = 10, collinearity 0.9, 1%
homoscedastic noise (seeded synthetic collinear-factor design), seeded U(0,1)
start.  A step is one ALS sweep of the mixed form: three MTTKRPs (FP32
matrix-core GEMM + FP64 Hadamard-reduce), three FP64 R x R Cholesky updates with
Gram/Hadamard products, normalization and the fused FP64 objective.  The tensor
and factors are resident in HBM before the timed region starts.

Reported (one JSON line on stdout):
  value            mixed-form ALS sweeps/s over the timed steps
  fp64_sweeps_per_s  the same sweep with every contraction in FP64
  roofline         the dominant MTTKRP kernel: algorithmic bytes per launch /
                   its average duration (HIP events on the library's stream)
  equal_fit        FP64 ALS and the mixed form (FP32 sweeps + FP64 refinement)
                   from the same start to a relative fit change of 1e-12
  cpu_baseline     the FP64 NumPy oracle's ALS sweep rate on the host (bounded sample)

Progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
PMC_SUMMARY = os.path.join(HERE, "profiles", "mttkrp_256cube_r10_pmc.md")
KERNEL_SOURCES = ["mttkrp.hip", "mttkrp_kernels.hpp", "mttkrp_k_f32v4.hip", "mttkrp_k_f32v8.hip",
                  "mttkrp_k_f64.hip", "sweep.hpp", "internal.hpp", "smallla.hpp"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "paper_1111_6091_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None
    when there is none or the kernel sources changed after the counters were taken."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    with open(PMC_SUMMARY) as f:
        for line in f:
            if line.startswith("traffic_json:"):
                t = json.loads(line.split(":", 1)[1])
                if t.get("source_hash") != kernel_source_hash():
                    return None
                return t.get("bytes_per_launch", {}).get(kernel)
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--workload", default="c3_256cube_r10")
    p.add_argument("--no-equal-fit", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-tune", action="store_true")
    p.add_argument("--no-multilevel", action="store_true",
                   help="skip the 128^3 R=5 CP-FAS leg (4 levels)")
    p.add_argument("--no-batched", action="store_true",
                   help="skip the batched leg (512 tensors x 4 restarts, mixed form)")
    p.add_argument("--plans-file", default=None,
                   help="import launch plans from this file instead of autotuning")
    p.add_argument("--save-plans", default=None, help="write the tuned launch plans to this file")
    p.add_argument("--mttkrp-only", action="store_true",
                   help="launch each MTTKRP kernel --steps times and a 64 MiB device copy "
                        "(byte-counter calibration), then exit; for profiler runs")
    p.add_argument("--vcycles-only", action="store_true",
                   help="time CP-FAS V-cycles on the 128^3 R=5 4-level hierarchy (FP64 and mixed, graph "
                        "replay off and on), then exit; for profiler runs")
    p.add_argument("--no-dense", action="store_true",
                   help="skip the Table 3/4 legs (dense (i^2+j^2+k^2)^(-1/2) and sparse Laplacian "
                        "tensors: Multilevel (+ FMG) vs ALS)")
    p.add_argument("--dense-only", action="store_true",
                   help="run only the Table 3/4 legs and print their JSON")
    p.add_argument("--restrict-only", action="store_true",
                   help="time only the coarse-tensor restrictions and print their JSON")
    p.add_argument("--batched-only", action="store_true",
                   help="run only the batched leg (512 problems x 4 restarts, mixed then FP64) and "
                        "print its JSON; for profiler runs")
    p.add_argument("--sweeps-only", action="store_true",
                   help="time the mixed and FP64 sweeps only, then exit; for profiler runs")
    p.add_argument("--cold", action="store_true",
                   help="with --mttkrp-only: write and read a 1 GiB buffer before every MTTKRP "
                        "launch (evicts the L2 caches and the 256 MB Infinity Cache)")
    return p.parse_args()


def mttkrp_bytes(dims, R, n, elem_bytes):
    """Algorithmic bytes of one MTTKRP: the tensor once, the other factors, the output."""
    P = math.prod(dims)
    other = sum(d for m, d in enumerate(dims) if m != n)
    return P * elem_bytes + other * R * elem_bytes + dims[n] * R * 8


def tree_y_doubles(dims, R, elem_bytes):
    """Entries of the stage-1 tiles Y = Z x_1 A^(1)T the sweep keeps (stored in the
    tensor's precision, elem_bytes each), or 0 when the sweep runs one pass over Z
    per mode (order 2, or Y in FP64 above a quarter of Z's bytes)."""
    if len(dims) < 3:
        return 0
    yd = math.prod(dims[2:]) * dims[1] * R
    return yd if yd * 8 * 4 <= math.prod(dims) * elem_bytes else 0


def sweep_mttkrp_bytes(dims, R, n, elem_bytes):
    """Algorithmic bytes of the sweep's mode-n launch: with the dimension tree,
    mode 1 also writes Y once and modes >= 2 read Y once (with the FP64 factors
    of modes 1.. other than n) instead of the tensor."""
    yd = tree_y_doubles(dims, R, elem_bytes)
    if yd == 0 or n == 0:
        return mttkrp_bytes(dims, R, n, elem_bytes)
    if n == 1:
        return mttkrp_bytes(dims, R, n, elem_bytes) + yd * elem_bytes
    other = sum(d for m, d in enumerate(dims) if m >= 1 and m != n)
    return yd * elem_bytes + other * R * 8 + dims[n] * R * 8


def sweep_mttkrp_overhead_bytes(dims, R, n, elem_bytes):
    """Bytes the sweep's mode-n launch moves beyond the algorithmic bytes of an
    MTTKRP: the mode-1 launch's Y store (the dimension tree's trade: written
    once, read by the modes >= 2 instead of another pass over Z)."""
    yd = tree_y_doubles(dims, R, elem_bytes)
    return yd * elem_bytes if (yd and n == 1) else 0


def sweep_kernel_name(dims, R, n, tag):
    """Name of the sweep's mode-n MTTKRP launch (matches the counter summary)."""
    tree = tree_y_doubles(dims, R, 4 if tag == "f32" else 8) > 0
    if tree and n >= 2:
        return "ymttkrp_modeN"
    if tree and n == 1:
        return f"mttkrp_mode1y_{tag}"
    return f"mttkrp_{('mode0', 'mode1', 'modeN')[min(n, 2)]}_{tag}"


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures the single-GPU kernel path only; run it with --gpus 1 "
              "(sharding over several GPUs is described in the design notes and not implemented)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1111_6091_amd import api, drivers, synth
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED, CP_SOLVE_CHOL

    torch.cuda.set_device(0)
    ctx = api.Context()
    K, W = args.steps, args.warmup
    if args.vcycles_only:
        vcycle_timing(ctx, api, drivers, synth)
        return
    if args.restrict_only:
        print(json.dumps({"restriction": restrict_leg(ctx, api, synth)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": batched_leg(ctx, api, synth)}), flush=True)
        return
    if args.dense_only:
        print(json.dumps({"dense_table4": dense_leg(ctx, api, drivers, synth),
                          "laplacian_table3": laplacian_leg(ctx, api, drivers, synth)}), flush=True)
        return
    Z, _, spec = synth.workload(args.workload)
    dims, R = tuple(spec["dims"]), spec["R"]
    A0 = synth.uniform_start(dims, R, spec["seed"])
    Zd = api.DeviceTensor.from_numpy(ctx, Z, fp32=True)
    torch.cuda.synchronize()
    log(f"workload {args.workload}: dims={dims} R={R}; tensor resident ({Z.nbytes / 1e6:.1f} MB FP64 "
        f"+ {Z.nbytes / 2e6:.1f} MB FP32)")

    def fresh():
        return api.DeviceFactors.from_numpy(ctx, A0, fp32=True)

    fh = torch.zeros(max(K, W, 1), dtype=torch.float64, device="cuda")

    # launch-configuration autotuner (before any timed region)
    plans = None
    if args.plans_file:
        with open(args.plans_file) as f:
            api.cp_plans_import(ctx, f.read())
        plans = api.cp_plans_export(ctx)
        log(f"plans imported from {args.plans_file}")
    elif not args.no_tune:
        t0 = time.perf_counter()
        At = fresh()
        for prec in (CP_MIXED, CP_FP64):
            api.cp_autotune(ctx, Zd, At, prec, 10)
        torch.cuda.synchronize()
        plans = api.cp_plans_export(ctx)
        log(f"autotune {time.perf_counter() - t0:.2f} s:\n{plans}")
    if args.save_plans and plans:
        with open(args.save_plans, "w") as f:
            f.write(plans)

    if args.mttkrp_only:
        # the sweep's launches (dimension tree), then one pass over Z per mode
        from paper_1111_6091_amd._lib import CP_OPT_DIMTREE
        A = fresh()
        flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda") if args.cold else None
        flush_sum = torch.empty(1, dtype=torch.float32, device="cuda")
        for tree in (1, 0):
            ctx.set_option(CP_OPT_DIMTREE, tree)
            for prec in (CP_MIXED, CP_FP64):
                for n in range(len(dims)):
                    if flush is None:
                        api.cp_time_mttkrp(ctx, Zd, A, n, prec, K)
                        continue
                    for _ in range(K):
                        flush.fill_(1.0)
                        torch.sum(flush, dim=0, keepdim=True, out=flush_sum)
                        api.cp_time_mttkrp(ctx, Zd, A, n, prec, 1)
        ctx.set_option(CP_OPT_DIMTREE, 1)
        src = torch.empty(64 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(K):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"mttkrp-only: {K} launches of each MTTKRP (dimension tree on and off, mixed and fp64, "
            f"{len(dims)} modes) and of a 64 MiB copy; kernel source hash {kernel_source_hash()}")
        return

    def timed(prec, steps, warm):
        A = fresh()
        if warm:
            api.cp_als_sweep(ctx, Zd, A, None, warm, CP_SOLVE_CHOL, 10, True, prec, fh)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        api.cp_als_sweep(ctx, Zd, A, None, steps, CP_SOLVE_CHOL, 10, True, prec, fh)
        e1.record()
        t_enq = time.perf_counter() - t0
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        timed.enqueue_us = t_enq / steps * 1e6
        return e0.elapsed_time(e1) / steps, wall

    ms_mixed, wall_mixed = timed(CP_MIXED, K, W)
    log(f"mixed sweep: {ms_mixed * 1e3:.1f} us ({1e3 / ms_mixed:.0f} sweeps/s; "
        f"host enqueue {timed.enqueue_us:.1f} us per sweep)")
    ms_fp64, wall_fp64 = timed(CP_FP64, K, W)
    log(f"fp64 sweep: {ms_fp64 * 1e3:.1f} us ({1e3 / ms_fp64:.0f} sweeps/s; "
        f"host enqueue {timed.enqueue_us:.1f} us per sweep)")
    if args.sweeps_only:
        return
    # the same sweeps with one pass over Z per mode (no dimension tree)
    from paper_1111_6091_amd._lib import CP_OPT_DIMTREE
    ctx.set_option(CP_OPT_DIMTREE, 0)
    ms_mixed_pm, _ = timed(CP_MIXED, K, W)
    ms_fp64_pm, _ = timed(CP_FP64, K, W)
    ctx.set_option(CP_OPT_DIMTREE, 1)
    log(f"per-mode MTTKRPs: mixed {ms_mixed_pm * 1e3:.1f} us, fp64 {ms_fp64_pm * 1e3:.1f} us per sweep")

    # roofline leg: each MTTKRP launch of the sweep timed over back-to-back
    # launches in the sweep's launch configuration (HIP events on the library's
    # stream); with the dimension tree, modes >= 2 are the launches contracting Y
    A = fresh()
    reps = max(10, min(K, 100))
    roof = {}
    for prec, tag, eb in ((CP_MIXED, "f32", 4), (CP_FP64, "f64", 8)):
        for n in range(len(dims)):
            ms = api.cp_time_mttkrp(ctx, Zd, A, n, prec, reps)
            ov = sweep_mttkrp_overhead_bytes(dims, R, n, eb)
            b = sweep_mttkrp_bytes(dims, R, n, eb) - ov
            roof[f"{tag}_mode{n}"] = dict(kernel=sweep_kernel_name(dims, R, n, tag),
                                          avg_us=ms * 1e3, bytes_per_launch=b, overhead_bytes=ov,
                                          achieved_gbs=b / (ms * 1e-3) / 1e9)
            log(f"{tag} mode {n}: {ms * 1e3:.2f} us/launch, {b / (ms * 1e-3) / 1e9:.0f} GB/s algorithmic"
                f" (+{ov / 1e6:.2f} MB overhead)")
    # cold launches: a 1 GiB buffer is written and then read before each launch,
    # so neither the L2 caches nor the 256 MB Infinity Cache hold the tensor
    # (the read leaves them clean: no write-back of the flush inside the timed
    # launch); single launches between their own events, median of 20, warm
    # single launches (the same method without the flush) beside them
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    flush_sum = torch.empty(1, dtype=torch.float32, device="cuda")

    def evict():
        flush.fill_(1.0)
        torch.sum(flush, dim=0, keepdim=True, out=flush_sum)

    cold = {}
    for prec, tag, eb in ((CP_MIXED, "f32", 4), (CP_FP64, "f64", 8)):
        for n in range(2):
            c_ms, w_ms = [], []
            for _ in range(20):
                evict()
                c_ms.append(api.cp_time_mttkrp(ctx, Zd, A, n, prec, 1))
                w_ms.append(api.cp_time_mttkrp(ctx, Zd, A, n, prec, 1))
            b = sweep_mttkrp_bytes(dims, R, n, eb) - sweep_mttkrp_overhead_bytes(dims, R, n, eb)
            cm, wm = float(np.median(c_ms)), float(np.median(w_ms))
            cold[f"{tag}_mode{n}"] = {"cold_us": round(cm * 1e3, 2), "warm_single_us": round(wm * 1e3, 2),
                                      "cold_gbs": round(b / (cm * 1e-3) / 1e9, 1),
                                      "cold_p10_p90_us": [round(float(np.percentile(c_ms, q)) * 1e3, 2)
                                                          for q in (10, 90)]}
            log(f"{tag} mode {n} cold: {cm * 1e3:.2f} us ({b / (cm * 1e-3) / 1e9:.0f} GB/s), "
                f"warm single launch {wm * 1e3:.2f} us")
    del flush
    torch.cuda.empty_cache()

    # per-kernel breakdown of one sweep (event pair around every launch)
    breakdown = {}
    for prec, tag in ((CP_MIXED, "f32"), (CP_FP64, "f64")):
        A = fresh()
        api.cp_als_sweep(ctx, Zd, A, None, 2, CP_SOLVE_CHOL, 10, True, prec, fh)
        ctx.profile(True)
        api.cp_als_sweep(ctx, Zd, A, None, K, CP_SOLVE_CHOL, 10, True, prec, fh)
        ctx.profile(False)
        breakdown[tag] = {k: round(v[0] / K * 1e3, 2) for k, v in ctx.profile_read().items()}
        log(f"{tag} per-sweep breakdown (us, event-bracketed): {breakdown[tag]}")
    mix = [v for k, v in roof.items() if k.startswith("f32_mode")]
    dom = max(mix, key=lambda v: v["avg_us"])
    roofline = {
        "bound": "hbm", "kernel": dom["kernel"], "achieved": round(dom["achieved_gbs"], 1),
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom["achieved_gbs"] / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(dom["kernel"]), "bytes_per_launch": dom["bytes_per_launch"],
        "overhead_bytes": dom["overhead_bytes"], "avg_launch_us": round(dom["avg_us"], 2),
        "bytes_note": "algorithmic bytes: the tensor once, the other factors, the output "
                      "(P*4 + sum_{m != n} I_m R 4 + I_n R 8); overhead_bytes: the Y store",
    }
    # the whole sweep against the dimension-tree bound: two passes over Z per sweep
    sweep_bytes = sum(r["bytes_per_launch"] for k, r in roof.items() if k.startswith("f32_"))
    sweep_roof = {"bytes_per_sweep": sweep_bytes,
                  "achieved_gbs": round(sweep_bytes / (ms_mixed * 1e-3) / 1e9, 1),
                  "frac": round(sweep_bytes / (ms_mixed * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "bound_sweeps_per_s": round(HBM_PEAK_GBS * 1e9 / sweep_bytes, 1),
                  "note": "sum of the algorithmic bytes of the sweep's MTTKRP launches (mode 0 and mode 1 "
                          "read Z, modes >= 2 read Y) over the measured mixed sweep time"}

    equal_fit = None
    if not args.no_equal_fit:
        A = fresh()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r64 = drivers.als_solve(ctx, Zd, A, max_sweeps=10000, fit_tol=1e-12, prec=CP_FP64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        fit64 = drivers.exact_fit(ctx, Zd, A)
        log(f"fp64 ALS to 1e-12: {r64.sweeps} sweeps, {t64:.3f} s, fit {fit64:.15f}")
        A = fresh()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rm = drivers.mixed_solve(ctx, Zd, A, tol32=1e-9, tol64=1e-12)
        torch.cuda.synchronize()
        tm = time.perf_counter() - t0
        fitm = drivers.exact_fit(ctx, Zd, A)
        log(f"mixed to 1e-12: {rm.sweeps32} FP32 + {rm.sweeps64} FP64 sweeps, {tm:.3f} s, fit {fitm:.15f}")
        equal_fit = {
            "stop": "relative fit change <= 1e-12 (FP32 phase: alarm at a mean FP32-objective gain <= 1e-9 "
                    "per sweep, then ends at a mean FP64-contraction fit gain <= 1e-11 per sweep over a "
                    "16-sweep chunk)",
            "fp64": {"sweeps": r64.sweeps, "seconds": round(t64, 4), "fit": fit64},
            "mixed": {"sweeps_fp32": rm.sweeps32, "sweeps_fp64": rm.sweeps64,
                      "seconds": round(tm, 4), "fit": fitm},
            "rel_fit_diff": abs(fitm - fit64) / abs(fit64),
            "speedup_mixed_vs_fp64": round(t64 / tm, 3) if tm > 0 else None,
        }
        gpath = os.path.join(HERE, "tests", "golden", f"als_{args.workload}.json")
        if os.path.exists(gpath):
            with open(gpath) as f:
                g = json.load(f)
            equal_fit["oracle_fit"] = g["final_fit_exact"]
            equal_fit["oracle_sweeps"] = g["sweeps"]
            equal_fit["fp64_rel_err_vs_oracle"] = abs(fit64 - g["final_fit_exact"]) / g["final_fit_exact"]
            equal_fit["mixed_rel_err_vs_oracle"] = abs(fitm - g["final_fit_exact"]) / g["final_fit_exact"]
            # parity at equal sweep counts: the FP64 path run for exactly the
            # oracle's sweeps (the 1e-12 rule can trip a few sweeps apart on two
            # trajectories that agree to rounding)
            A = fresh()
            done = 0
            while done < g["sweeps"]:
                k = min(256, g["sweeps"] - done)
                api.cp_als_sweep(ctx, Zd, A, None, k, CP_SOLVE_CHOL, 10, True, CP_FP64)
                done += k
            fit_eq = drivers.exact_fit(ctx, Zd, A)
            equal_fit["fp64_at_oracle_sweeps"] = {
                "sweeps": g["sweeps"], "fit": fit_eq,
                "rel_err_vs_oracle": abs(fit_eq - g["final_fit_exact"]) / g["final_fit_exact"]}
            log(f"fp64 at the oracle's {g['sweeps']} sweeps: fit {fit_eq:.16f}, rel err "
                f"{abs(fit_eq - g['final_fit_exact']) / g['final_fit_exact']:.2e}")

    batched = None
    if not args.no_batched:
        batched = batched_leg(ctx, api, synth)

    multilevel = None
    order4 = None
    restriction = None
    if not args.no_multilevel:
        restriction = restrict_leg(ctx, api, synth)
        multilevel = fas_leg(ctx, api, drivers, synth)
        order4 = order4_leg(ctx, api, drivers, synth, K)
    dense = laplacian = None
    if not args.no_dense:
        dense = dense_leg(ctx, api, drivers, synth)
        laplacian = laplacian_leg(ctx, api, drivers, synth)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(Z, A0, args.cpu_seconds)
        log(f"cpu oracle: {cpu['value']:.2f} sweeps/s on {cpu['cores']} threads")

    value = 1e3 / ms_mixed
    out = {
        "metric": "MTTKRP HBM GB/s + ALS sweeps/s, 256^3 R=10; mixed vs FP64 at equal fit",
        "value": round(value, 2),
        "unit": "ALS sweeps/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(ms_mixed, 5),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32 (MFMA contractions) + f64",
        "data": "synthetic",
        "config": {"workload": f"dense {dims[0]}x{dims[1]}x{dims[2]}, R={R}, collinearity "
                               f"{spec['c']}, noise {spec['eta_h']}, mixed FP32/FP64 ALS sweep",
                   "dims": list(dims), "rank": R, "parallelism": "single GPU"},
        "fp64_sweeps_per_s": round(1e3 / ms_fp64, 2),
        "sweep_us": {"mixed": round(ms_mixed * 1e3, 2), "fp64": round(ms_fp64 * 1e3, 2),
                     "mixed_per_mode_passes": round(ms_mixed_pm * 1e3, 2),
                     "fp64_per_mode_passes": round(ms_fp64_pm * 1e3, 2),
                     "note": "default sweeps stream Z twice (mode 0, mode 1 + stage-1 tiles reused by "
                             "mode 2); per_mode_passes stream Z once per mode"},
        "wall_seconds": {"mixed": round(wall_mixed, 4), "fp64": round(wall_fp64, 4)},
        "mttkrp_gbs": {k: round(v["achieved_gbs"], 1) for k, v in roof.items()},
        "mttkrp_us": {k: round(v["avg_us"], 2) for k, v in roof.items()},
        "roofline": roofline,
        "sweep_roofline": sweep_roof,
        "mttkrp_cold": cold,
        "per_sweep_us_event_bracketed": breakdown,
        "equal_fit": equal_fit,
        "tuned_plans": plans.strip().splitlines() if plans else None,
        "batched": batched,
        "multilevel_128cube_r5": multilevel,
        "order4_64quart_r8": order4,
        "restriction": restriction,
        "dense_table4": dense,
        "laplacian_table3": laplacian,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def fas_leg(ctx, api, drivers, synth):
    """128^3 R=5 (c = 0.9, 1% + 1% noise), FP64: CP-FAS V-cycles (Algorithm 2, Table 1
    parameters) on the 4-level hierarchy from the oracle's setup phase (stored
    interpolation weights and setup factors, an input here) against standalone ALS
    from the same factors, each to a relative fit change of 1e-12."""
    import numpy as np
    import torch
    path = os.path.join(HERE, "tests", "golden", "fas_c2_128cube_r5.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    Z, _, spec = synth.workload("c2_128cube_r5")
    weights = [[None if w is None else np.asarray(w) for w in lv] for lv in g["weights"]]
    Zd = api.DeviceTensor.from_numpy(ctx, Z)
    levels = drivers.build_hierarchy(ctx, Zd, weights)
    A0 = [np.asarray(a) for a in g["A_setup"]]
    out = {"levels": len(levels), "coarsest": g["coarsest"], "stop": "relative fit change <= 1e-12",
           "oracle": {"fas_cycles": g["fas_cycles"], "fas_fit": g["fas_fit"], "fas_seconds": round(g["fas_seconds"], 1),
                      "als_sweeps": g.get("als_sweeps"), "als_fit": g.get("als_fit"),
                      "als_seconds": round(g.get("als_seconds", 0.0), 1)}}
    A = api.DeviceFactors.from_numpy(ctx, A0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = drivers.fas_solve(ctx, levels, Zd, A, fit_tol=1e-12, nu1=1, nu2=1, nuc=50, gs_iters=10)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    A = api.DeviceFactors.from_numpy(ctx, A0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ra = drivers.als_solve(ctx, Zd, A, fit_tol=1e-12, prec=0, sort_at_end=False)
    torch.cuda.synchronize()
    ta = time.perf_counter() - t0
    fit_als = drivers.exact_fit(ctx, Zd, A)
    out["fas"] = {"cycles": r.sweeps, "seconds": round(tf, 4), "ms_per_cycle": round(1e3 * tf / r.sweeps, 3),
                  "fit": r.final_fit,
                  "rel_fit_err_vs_oracle": abs(r.final_fit - g["fas_fit"]) / abs(g["fas_fit"]),
                  "ms_per_cycle_by_level": fas_cost_by_level(ctx, api, synth, levels)}
    out["als"] = {"sweeps": ra.sweeps, "seconds": round(ta, 4), "us_per_sweep": round(1e6 * ta / ra.sweeps, 1),
                  "fit": fit_als}
    if g.get("als_fit"):
        out["als"]["rel_fit_err_vs_oracle"] = abs(fit_als - g["als_fit"]) / abs(g["als_fit"])
    log(f"128^3 FAS: {r.sweeps} V-cycles in {tf:.3f} s ({1e3 * tf / r.sweeps:.2f} ms/cycle), fit {r.final_fit:.13f}; "
        f"ALS: {ra.sweeps} sweeps in {ta:.3f} s, fit {fit_als:.13f}; ms per cycle by level "
        f"{[lv['ms'] for lv in out['fas']['ms_per_cycle_by_level']]}")
    return out


def fas_cost_by_level(ctx, api, synth, levels, cycles=20):
    """Cost of one V-cycle by level.  t_k: a cycle on the hierarchy from level k
    down (level k then takes the finest level's place, without a right-hand
    side), for every k with a coarser level below it; the coarsest level's
    share is its nu_c = 50 Gauss-Seidel sweeps as the cycle runs them (one
    workgroup).  Level k's share is t_k - t_(k+1), the last intermediate
    level's t_k minus the coarsest share.  Factors of level k: 5 FP64 ALS
    sweeps from a seeded start on that level's tensor."""
    import torch

    def timed(fn):
        fn()   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(cycles):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / cycles

    def factors(k):
        Zk = levels[k][0]
        A = api.DeviceFactors.from_numpy(ctx, synth.uniform_start(tuple(Zk.dims), 5, 11))
        api.cp_als_sweep(ctx, Zk, A, None, 5, api.CP_SOLVE_CHOL, 10, True, api.CP_FP64)
        return A

    L = len(levels)
    t = []
    for k in range(L - 1):
        A = factors(k)
        t.append(timed(lambda: api.cp_fas_vcycle(ctx, levels[k:], A, nu1=1, nu2=1, nuc=50, gs_iters=10)))
    A = factors(L - 1)
    coarse = timed(lambda: api.cp_als_sweep(ctx, levels[-1][0], A, None, 50, api.CP_SOLVE_GS, 10, False,
                                            api.CP_FP64))
    share = [t[k] - t[k + 1] for k in range(L - 2)] + [t[L - 2] - coarse, coarse]
    return [{"level": k, "dims": [int(d) for d in levels[k][0].dims], "ms": round(share[k], 3)}
            for k in range(L)]


# Table 4 (dense problem, averages over the paper's successful runs; MATLAB on a
# 2.5 GHz Core 2 Duo): test -> ALS iterations, ALS seconds, Multilevel + FMG
# iterations, seconds, levels.
TABLE4 = {2: dict(als_it=2435, als_s=11.8, ml_it=15, ml_s=2.7, levs=5),
          6: dict(als_it=1695, als_s=80.2, ml_it=9, ml_s=8.1, levs=6)}


def dense_leg(ctx, api, drivers, synth, tests=(2, 6)):
    """Section 6.3's dense tensor (i^2+j^2+k^2)^(-1/2), FP64, first seeded run of
    Table 4's tests: 'Multilevel + FMG' (Section 6.1, Table 1 parameters) and
    standalone ALS from the same boot factors, both to g < 1e-10 (eq. (31)).
    The multilevel time includes its g evaluations (they drive the stagnation
    rules); the ALS time is that of exactly the sweep count found by a first run
    with g after every sweep (the paper's times leave the stopping test out)."""
    import torch
    out = []
    for t in tests:
        s, R = synth.DENSE_TESTS[t]
        d = synth.dense_case(s, R)
        Zd = api.DeviceTensor.from_numpy(ctx, d["Z"])
        cdims = [s] * 3
        while any(x > d["coarsest"][n] for n, x in enumerate(cdims)):
            cdims = [(x + 1) // 2 if x > d["coarsest"][n] else x for n, x in enumerate(cdims)]
        cs = synth.dense_coarse_start(cdims, R, d["seed"])
        A = api.DeviceFactors.from_numpy(ctx, d["boot"])
        T = [api.DeviceFactors.from_numpy(ctx, x) for x in d["tfms"]]
        Cd = api.DeviceFactors.from_numpy(ctx, cs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = drivers.multilevel_fmg(ctx, Zd, A, T, d["coarsest"], Cd,
                                      fas=dict(nu1=1, nu2=1, nuc=50, gs_iters=10))
        torch.cuda.synchronize()
        t_ml = time.perf_counter() - t0
        fit_ml = drivers.exact_fit(ctx, Zd, A)
        B = api.DeviceFactors.from_numpy(ctx, d["boot"])
        sweeps, gh = drivers.als_solve_g(ctx, Zd, B, tau=1e-10, max_sweeps=10000)
        fit_als = drivers.exact_fit(ctx, Zd, B)
        B = api.DeviceFactors.from_numpy(ctx, d["boot"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.cp_als_sweep(ctx, Zd, B, None, sweeps, 0, 10, True, 0)
        torch.cuda.synchronize()
        t_als = time.perf_counter() - t0
        row = {"test": t, "s": s, "R": R, "levels": info["levels"],
               "multilevel_fmg": {"iterations": info["iterations"], "setup_cycles": len(info["setup"]),
                                  "solve_cycles": len(info["solve"]), "rebuilt": info["rebuilt"],
                                  "g": info["solve"][-1] if info["solve"] else None,
                                  "seconds": round(t_ml, 4), "fit": fit_ml},
               "als": {"sweeps": sweeps, "converged": bool(gh and gh[-1] < 1e-10), "g": gh[-1] if gh else None,
                       "seconds": round(t_als, 4), "us_per_sweep": round(1e6 * t_als / max(sweeps, 1), 1),
                       "fit": fit_als},
               "speedup": round(t_als / t_ml, 3),
               "paper_table4": TABLE4.get(t)}
        log(f"dense test {t} (s={s}, R={R}, {info['levels']} levels): Multilevel+FMG {info['iterations']} it "
            f"in {t_ml:.3f} s; ALS {sweeps} sweeps in {t_als:.3f} s; speedup {t_als / t_ml:.2f}")
        out.append(row)
    return out


# Table 3 (sparse problem; same machine and averaging as Table 4): test -> ALS
# iterations and seconds, Multilevel and Multilevel + FMG iterations and
# seconds, levels.
TABLE3 = {1: dict(als_it=1897, als_s=24.0, ml_it=37, ml_s=7.6, fmg_it=36, fmg_s=8.0, levs=2),
          5: dict(als_it=5508, als_s=150.3, ml_it=182, ml_s=64.9, fmg_it=99, fmg_s=40.9, levs=4),
          8: dict(als_it=3481, als_s=610.0, ml_it=72, ml_s=164.8, fmg_it=70, fmg_s=177.9, levs=3),
          11: dict(als_it=1743, als_s=943.3, ml_it=39, ml_s=402.3, fmg_it=43, fmg_s=474.0, levs=3)}


def laplacian_leg(ctx, api, drivers, synth, tests=(1, 5, 8, 11)):
    """Section 6.2's sparse Laplacian tensors (the finest level in the sparse
    form, coarse levels dense), FP64, first seeded run of Table 3's tests:
    'Multilevel' and 'Multilevel + FMG' (Section 6.1, Table 1 parameters) and
    standalone ALS from the same boot factors, all to g < 1e-10 (eq. (31)),
    timed as in the dense leg."""
    import torch
    fas = dict(nu1=1, nu2=1, nuc=50, gs_iters=10)
    out = []
    for t in tests:
        N, s, R = synth.LAPLACIAN_TESTS[t]
        c = synth.laplacian_case(N, s, R)
        Zs = api.SparseTensor.from_coo(ctx, c["idx"], c["vals"], c["shape"])
        cdims = [s] * N
        while any(x > c["coarsest"][n] for n, x in enumerate(cdims)):
            cdims = [(x + 1) // 2 if x > c["coarsest"][n] else x for n, x in enumerate(cdims)]
        row = {"test": t, "N": N, "s": s, "R": R, "nnz": int(c["vals"].shape[0])}
        for name, fmg in (("multilevel", False), ("multilevel_fmg", True)):
            A = api.DeviceFactors.from_numpy(ctx, c["boot"])
            T = [api.DeviceFactors.from_numpy(ctx, x) for x in c["tfms"]]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if fmg:
                Cd = api.DeviceFactors.from_numpy(ctx, synth.dense_coarse_start(cdims, R, c["seed"]))
                info = drivers.multilevel_fmg(ctx, Zs, A, T, c["coarsest"], Cd, fas=fas)
            else:
                info = drivers.multilevel(ctx, Zs, A, T, c["coarsest"], fas=fas)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            row["levels"] = info["levels"]
            row[name] = {"iterations": info["iterations"], "setup_cycles": len(info["setup"]),
                         "solve_cycles": len(info["solve"]), "rebuilt": info["rebuilt"],
                         "converged": bool(info["solve"] and info["solve"][-1] < 1e-10),
                         "seconds": round(el, 4), "fit": drivers.exact_fit(ctx, Zs, A)}
        B = api.DeviceFactors.from_numpy(ctx, c["boot"])
        sweeps, gh = drivers.als_solve_g(ctx, Zs, B, tau=1e-10, max_sweeps=10000)
        fit_als = drivers.exact_fit(ctx, Zs, B)
        B = api.DeviceFactors.from_numpy(ctx, c["boot"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.cp_als_sweep(ctx, Zs, B, None, sweeps, 0, 10, True, 0)
        torch.cuda.synchronize()
        t_als = time.perf_counter() - t0
        row["als"] = {"sweeps": sweeps, "converged": bool(gh and gh[-1] < 1e-10), "seconds": round(t_als, 4),
                      "us_per_sweep": round(1e6 * t_als / max(sweeps, 1), 1), "fit": fit_als}
        row["speedup"] = {k: round(t_als / row[k]["seconds"], 3) for k in ("multilevel", "multilevel_fmg")}
        row["paper_table3"] = TABLE3.get(t)
        log(f"laplacian test {t} (N={N}, s={s}, R={R}, nnz={row['nnz']}, {row['levels']} levels): "
            f"Multilevel {row['multilevel']['iterations']} it {row['multilevel']['seconds']:.3f} s; "
            f"+FMG {row['multilevel_fmg']['iterations']} it {row['multilevel_fmg']['seconds']:.3f} s; "
            f"ALS {sweeps} sweeps {t_als:.3f} s")
        out.append(row)
    return out


def restrict_leg(ctx, api, synth, reps=20):
    """Coarse-tensor construction eq. (15) as dense P^T GEMMs on the matrix
    cores, every mode coarsened: 256^3 -> 128^3 (FP32, the 256^3 tensor's
    shadow) and 128^3 -> 64^3 (FP64), linear-interpolation P^.  Algorithmic
    flops: sum over modes of 2 I_c I (rest of the current tensor); algorithmic
    bytes: each mode product reads its input and writes its output once."""
    import numpy as np
    import torch
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED
    out = {}
    for name, prec, b, peak in (("c3_256cube_r10", CP_MIXED, 4, 157.3), ("c2_128cube_r5", CP_FP64, 8, 78.6)):
        Z, _, spec = synth.workload(name)
        dims = list(Z.shape)
        Zd = api.DeviceTensor.from_numpy(ctx, Z, fp32=prec == CP_MIXED)
        phat = []
        for d in dims:
            w = torch.from_numpy(synth.linear_interp_weights(d)).cuda()
            ph = torch.empty((d, (d + 1) // 2), dtype=torch.float64, device="cuda")
            api.cp_transfer_build(ctx, w, ph)
            phat.append(ph)
        cdims = [(d + 1) // 2 for d in dims]
        Zc = api.DeviceTensor.empty(cdims, fp64=prec == CP_FP64, fp32=prec == CP_MIXED)
        flops, byts, cur = 0.0, 0.0, list(dims)
        for n in range(len(dims)):
            rest = float(np.prod(cur)) / cur[n]
            flops += 2.0 * cdims[n] * cur[n] * rest
            byts += b * (np.prod(cur) + cdims[n] * rest)
            cur[n] = cdims[n]
        wd = [torch.from_numpy(synth.linear_interp_weights(d)).cuda() for d in dims]

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(reps):
                fn()
            e1.record(st)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) * 1e3 / reps

        us = timed(lambda: api.cp_restrict(ctx, Zd, phat, Zc, prec))
        usf = timed(lambda: api.cp_restrict_factored(ctx, Zd, wd, Zc, prec))
        tf = flops / (us * 1e-6) / 1e12
        out[name] = {"dims": dims, "coarse": cdims, "prec": "mixed (FP32 storage)" if prec == CP_MIXED else "fp64",
                     "dense_gemm": {"us": round(us, 2), "gflop": round(flops / 1e9, 3), "tflops": round(tf, 2),
                                    "frac_of_mfma_peak": round(tf / peak, 4),
                                    "gbs": round(byts / (us * 1e-6) / 1e9, 1)},
                     "factored": {"us": round(usf, 2), "gbs": round(byts / (usf * 1e-6) / 1e9, 1),
                                  "frac_of_hbm_peak": round(byts / (usf * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
                     "mb": round(byts / 1e6, 1),
                     "note": "mb: each mode product reads its input and writes its output once; the dense "
                             "form does 2 I_c flops per input entry (matrix cores), the factored form about 5 "
                             "flops per coarse entry (HBM-bound)"}
        log(f"restriction {name}: dense GEMM {us:.1f} us ({tf:.1f} TFLOP/s, {tf / peak:.3f} of {peak}), "
            f"factored {usf:.1f} us ({byts / (usf * 1e-6) / 1e9:.0f} GB/s)")
    return out


def vcycle_timing(ctx, api, drivers, synth, cycles=50):
    """ms per CP-FAS V-cycle on the 128^3 R=5 4-level hierarchy of the oracle's
    setup phase, FP64 and mixed, with the graph replay off and on (one untimed
    cycle first in each case)."""
    import numpy as np
    import torch
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED, CP_OPT_GRAPHS
    with open(os.path.join(HERE, "tests", "golden", "fas_c2_128cube_r5.json")) as f:
        g = json.load(f)
    Z, _, spec = synth.workload("c2_128cube_r5")
    Zd = api.DeviceTensor.from_numpy(ctx, Z, fp32=True)
    weights = [[None if w is None else np.asarray(w) for w in lv] for lv in g["weights"]]
    levels = drivers.build_hierarchy(ctx, Zd, weights, prec=CP_MIXED, fp32=True, fp64=True)
    A0 = [np.asarray(a) for a in g["A_setup"]]
    out = {}
    for graphs in (0, 1):
        ctx.set_option(CP_OPT_GRAPHS, graphs)
        for prec, tag in ((CP_FP64, "fp64"), (CP_MIXED, "mixed")):
            A = api.DeviceFactors.from_numpy(ctx, A0, fp32=True)
            api.cp_fas_vcycle(ctx, levels, A, prec=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(cycles):
                api.cp_fas_vcycle(ctx, levels, A, prec=prec)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / cycles * 1e3
            out[f"{tag}_graphs{graphs}"] = round(ms, 3)
            log(f"V-cycle {tag}, graph replay {graphs}: {ms:.3f} ms")
    ctx.set_option(CP_OPT_GRAPHS, 1)
    return out


def order4_leg(ctx, api, drivers, synth, steps):
    """64^4 R=8 (c = 0.8, 0.5% noise): ALS sweeps in both forms, each mode's MTTKRP,
    and CP-FAS V-cycles on the 3-level hierarchy (64 -> 32 -> 16) of the oracle's
    setup phase (stored weights and factors, an input here), mixed and FP64."""
    import numpy as np
    import torch
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED, CP_SOLVE_CHOL
    Z, _, spec = synth.workload("c4_64quart_r8")
    dims, R = tuple(spec["dims"]), spec["R"]
    A0 = synth.uniform_start(dims, R, spec["seed"])
    Zd = api.DeviceTensor.from_numpy(ctx, Z, fp32=True)
    At = api.DeviceFactors.from_numpy(ctx, A0, fp32=True)
    for prec in (CP_MIXED, CP_FP64):
        api.cp_autotune(ctx, Zd, At, prec, 10)
    out = {"dims": list(dims), "rank": R}
    fh = torch.zeros(steps, dtype=torch.float64, device="cuda")
    for prec, tag in ((CP_MIXED, "mixed"), (CP_FP64, "fp64")):
        A = api.DeviceFactors.from_numpy(ctx, A0, fp32=True)
        api.cp_als_sweep(ctx, Zd, A, None, 10, CP_SOLVE_CHOL, 10, True, prec, fh)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        api.cp_als_sweep(ctx, Zd, A, None, steps, CP_SOLVE_CHOL, 10, True, prec, fh)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[f"{tag}_sweep_us"] = round(ms * 1e3, 2)
        out[f"{tag}_sweeps_per_s"] = round(1e3 / ms, 1)
        eb = 4 if prec == CP_MIXED else 8
        out[f"{tag}_mttkrp_gbs"] = []
        out[f"{tag}_mttkrp_us"] = []
        for n in range(4):
            t = api.cp_time_mttkrp(ctx, Zd, A, n, prec, 50)
            out[f"{tag}_mttkrp_us"].append(round(t * 1e3, 2))
            out[f"{tag}_mttkrp_gbs"].append(round(sweep_mttkrp_bytes(dims, R, n, eb) / (t * 1e-3) / 1e9, 1))
    path = os.path.join(HERE, "tests", "golden", "fas_c4_64quart_r8.json")
    if os.path.exists(path):
        with open(path) as f:
            g = json.load(f)
        weights = [[None if w is None else np.asarray(w) for w in lv] for lv in g["weights"]]
        levels = drivers.build_hierarchy(ctx, Zd, weights, prec=CP_MIXED, fp32=True)
        fas = {"levels": len(levels), "oracle_fits_3_cycles": g["fas_fits"]}
        for prec, tag in ((CP_MIXED, "mixed"), (CP_FP64, "fp64")):
            A = api.DeviceFactors.from_numpy(ctx, [np.asarray(a) for a in g["A_setup"]], fp32=True)
            fits = []
            for _ in range(3):
                api.cp_fas_vcycle(ctx, levels, A, prec=prec)
                fits.append(drivers.exact_fit(ctx, Zd, A))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                api.cp_fas_vcycle(ctx, levels, A, prec=prec)
            torch.cuda.synchronize()
            fas[tag] = {"ms_per_cycle": round((time.perf_counter() - t0) * 1e2, 3), "fits_3_cycles": fits,
                        "max_rel_fit_err_vs_oracle": max(abs(a - b) / abs(b) for a, b in zip(fits, g["fas_fits"]))}
        out["fas_3_levels"] = fas
    log(f"64^4 R=8: mixed sweep {out['mixed_sweep_us']} us, fp64 sweep {out['fp64_sweep_us']} us; "
        f"MTTKRP GB/s mixed {out['mixed_mttkrp_gbs']} fp64 {out['fp64_mttkrp_gbs']}; FAS {out.get('fas_3_levels')}")
    return out


def batched_leg(ctx, api, synth):
    """512 collinear-factor tensors (modes 16..96, R 2..8, c in [0.3, 0.95]), 4 restarts
    each, mixed form to the 1e-12 rule (FP32 windows of 16 sweeps, gain 1e-9), then the
    same batch in FP64 only; every restart capped at 10000 sweeps."""
    import numpy as np
    import torch
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED
    probs = synth.batched_problems(512)
    P = np.array([float(np.prod(p["dims"])) for p in probs])
    out = {"problems": len(probs), "restarts": 4, "solves": 4 * len(probs),
           "entries_total": int(P.sum()), "cap_sweeps": 10000}
    for prec, tag in ((CP_MIXED, "mixed"), (CP_FP64, "fp64")):
        mixed = prec == CP_MIXED
        dev = []
        for p in probs:
            Zd = api.DeviceTensor.from_numpy(ctx, p["Z"], fp32=mixed)
            cat = [np.hstack([p["starts"][k][n] for k in range(4)]) for n in range(3)]
            dev.append((Zd, api.DeviceFactors.from_numpy(ctx, cat, fp32=mixed)))
        # launch tiles: tensor KiB per streaming workgroup, tuned on the first sweeps
        from paper_1111_6091_amd import drivers
        kib, tune_t = drivers.tune_batched(ctx, dev, 4, prec)
        log(f"batched {tag}: tile tuner {', '.join(f'{k} KiB {v * 1e3:.1f} ms' for k, v in tune_t.items())} "
            f"-> {kib} KiB")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fits, sweeps = api.cp_als_batched(ctx, dev, 4, prec=prec, window32=16, tol32=1e-9, tol64=1e-12,
                                          max_sweeps=10000, chunk=16, wg_kib=kib)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sw = sweeps.cpu().numpy()
        f = fits.cpu().numpy()
        # algorithmic bytes: N = 3 passes over each tensor per shared sweep
        shared32 = sw[:, :, 0].max(axis=1)
        shared64 = sw[:, :, 1].max(axis=1)
        byt = float((3 * P * 4 * shared32 + 3 * P * 8 * shared64).sum())
        # the same batch once more, every restart capped at the largest sweep
        # count of a restart that converged: the time without the capped tail
        tot = sw.sum(axis=2)
        uncapped = tot[tot < 10000]
        t_nocap = None
        if uncapped.size and (tot >= 10000).any():
            dev2 = []
            for p in probs:
                cat = [np.hstack([p["starts"][k][n] for k in range(4)]) for n in range(3)]
                dev2.append((dev[len(dev2)][0], api.DeviceFactors.from_numpy(ctx, cat, fp32=mixed)))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            api.cp_als_batched(ctx, dev2, 4, prec=prec, window32=16, tol32=1e-9, tol64=1e-12,
                               max_sweeps=int(uncapped.max()), chunk=16, wg_kib=kib)
            torch.cuda.synchronize()
            t_nocap = time.perf_counter() - t0
            del dev2
        out[tag] = {"seconds": round(dt, 4), "solves_per_s": round(4 * len(probs) / dt, 1),
                    "tuned_wg_kib": kib, "tuner_ms_per_8_sweeps": {str(k): round(v * 1e3, 2) for k, v in tune_t.items()},
                    "seconds_capped_at_max_converged_sweeps": None if t_nocap is None else round(t_nocap, 4),
                    "capped_tail_seconds": None if t_nocap is None else round(dt - t_nocap, 4),
                    "sweeps_fp32": int(sw[:, :, 0].sum()), "sweeps_fp64": int(sw[:, :, 1].sum()),
                    "max_sweeps_one_restart": int(sw.sum(axis=2).max()),
                    "restarts_at_cap": int((sw.sum(axis=2) >= 10000).sum()),
                    "algorithmic_gb": round(byt / 1e9, 2), "achieved_gbs": round(byt / dt / 1e9, 1),
                    "fit_median": float(np.median(f)), "fits": f}
        log(f"batched {tag}: {dt:.3f} s, {4 * len(probs) / dt:.0f} solves/s, "
            f"{byt / dt / 1e9:.0f} GB/s algorithmic, status {ctx.status()}")
        del dev
        torch.cuda.empty_cache()
    fm, f64 = out["mixed"].pop("fits"), out["fp64"].pop("fits")
    d = np.abs(fm - f64) / np.abs(f64)
    out["mixed_vs_fp64_rel_fit_diff"] = {"median": float(np.median(d)), "max": float(d.max()),
                                         "frac_within_1e-10": float((d <= 1e-10).mean())}
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(Z, A0, seconds):
    """The oracle's ALS sweep on the host: as many sweeps as fit in ``seconds`` with
    the BLAS thread pool as it is, then a third of that with one thread."""
    from oracle import cp
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count()

    def run(limit_s):
        A = [a.copy() for a in A0]
        t0 = time.perf_counter()
        n = 0
        while True:
            A = cp.als_sweep(Z, A)
            n += 1
            el = time.perf_counter() - t0
            if el >= limit_s or n >= 500:
                return n, el

    n, el = run(seconds)
    out = {"value": round(n / el, 3), "unit": "ALS sweeps/s", "cores": threads, "kind": "oracle",
           "sample": f"{n} FP64 NumPy oracle ALS sweeps (explicit Khatri-Rao MTTKRP) on the same "
                     f"{'x'.join(map(str, Z.shape))} R={A0[0].shape[1]} tensor from the same start, "
                     f"{el:.1f} s", "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            n1, el1 = run(seconds / 3)
        out["one_thread"] = {"value": round(n1 / el1, 3), "sample": f"{n1} sweeps, {el1:.1f} s"}
    return out


if __name__ == "__main__":
    main()
