"""Benchmark: the 2D single-grid suite on one MI355X.

Workload (one "step"): the four 2D stencils of the single-grid suite, each run
for T = 1000 steps on an 8192 x 8192 FP64 interior with a Dirichlet halo:
5-point star r=1, 9-point box r=1, 13-point star r=3, 25-point box r=2;
coefficients U[0,1) normalised to sum 1, inputs U[0,1) (seeded, synthetic).
Inputs are resident in HBM before timing starts.

Prints one JSON line: GCells/s over the whole step (cell-updates per second),
the roofline record of the dominant kernel (HBM or VALU, whichever bounds it),
the per-stencil breakdown with the fraction of the temporally blocked roofline
min(t_eff * B / 2S, F / 2k), and the CPU oracle timed on a bounded sample of
the same workload. Unless --no-extras is given, the same line also reports the
other workloads once each: the plain one-step kernel's rate, one grid-wide
barrier's cost, the suite in persistent launches and with autotuned plans,
the attainable-performance model next to each measured rate, the paper's
benchmark stencils at its domain sizes, the small Jacobi latency, the 3D
single-grid suite (512^3, T=200, FP64), the heterogeneous batch of 128 grids
in one persistent launch per dtype (FP64 and FP32, with the FP32 error against
the FP64 result and the fraction of its bytes/flops bound) and the serving
loop under Poisson arrivals (FP32, 200 warm-up + measured requests, p50/p99
latency from each request's scheduled arrival, an FP32 error sample, FP64
plain throughput, the same arrivals with two rounds in flight, a saturation
sweep (400-1600 req/s) that gives the served capacity, and a small-budget
stress run). The 3D rows carry device tiling's
best measured rate next to the overlapped tiles the planner picks.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 8192] [--T 1000]
                       [--no-cpu] [--no-extras] [--serve-seconds S]
       python bench.py --probe | --probe3d | --probe-batch   (short programs for
                       rocprofv3 counter and trace passes)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VALU_TFLOPS = 78.6
# FP32 as built: packed FP32 is not used, so FP32 FMAs issue at the FP64 rate
FP32_VALU_TFLOPS = 78.6
# resident requests of the serving runs: a round's work list holds one quantum
# of each, and with 64 the rounds of a loaded server had too few items to fill
# the device (served FP32 422 GCells/s at 1600 req/s against 630 with 256);
# at 200 req/s fewer than 20 are ever resident
SERVE_SLOTS = 256


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def copy_bandwidth_probe(stencil, nbytes=2 << 30):
    """Streaming-copy bandwidth of the library's own probe (128-bit loads and
    stores, best of its kernel variants), read + write bytes / s, GB/s."""
    return stencil.stencil_probe_copy(nbytes) / 1e9


def copy_bandwidth(torch, nbytes=2 << 30, reps=5):
    """torch's device-to-device copy (read + write bytes / time), GB/s; for
    comparison with the library's probe."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / best / 1e9


def cpu_baseline(problems, fields, budget_s=15.0):
    """Oracle on a bounded sample: every stencil of the suite on the full-size
    grid for a few steps, sized from a one-step calibration."""
    import oracle
    threads = oracle.default_threads()
    per_step = 0.0
    for prob, u0 in zip(problems, fields):
        t0 = time.perf_counter()
        oracle.sweep(prob.coeffs, prob.spec.r, u0, 1, threads=threads)
        t1 = time.perf_counter()
        oracle.sweep(prob.coeffs, prob.spec.r, u0, 3, threads=threads)
        t2 = time.perf_counter()
        per_step += max((t2 - t1) - (t1 - t0), 1e-3) / 2
    # the calibration overestimates a step (thread start-up), so the sample is
    # topped up from its own rate until it fills at least 2/3 of the budget
    steps, updates, dt = 0, 0, 0.0
    while steps < 1000 and dt < 0.67 * budget_s:
        est = dt / steps if steps else per_step
        n = max(1, min(1000 - steps, int((budget_s - dt) / max(est, 1e-3))))
        t0 = time.perf_counter()
        for prob, u0 in zip(problems, fields):
            oracle.sweep(prob.coeffs, prob.spec.r, u0, n, threads=threads)
            updates += prob.cells * n
        dt += time.perf_counter() - t0
        steps += n
    # one thread on the small Jacobi case (256^2 5-point, T = 16)
    from paper_2305_07390_amd import workloads
    small = workloads.small_jacobi_problem()
    su0 = small.field()
    oracle.sweep(small.coeffs, 1, su0, 1, threads=1)
    t1 = time.perf_counter()
    oracle.sweep(small.coeffs, 1, su0, small.T, threads=1)
    t1 = time.perf_counter() - t1
    return {
        "value": updates / dt / 1e9,
        "unit": "GCells/s",
        "cores": threads,
        "kind": "oracle",
        "one_thread_small_jacobi": {"gcells_per_s": round(small.updates / t1 / 1e9, 3), "ms": round(t1 * 1e3, 2),
                                    "workload": "256x256 5-point Jacobi, T=16, FP64, 1 thread"},
        "sample": f"all {len(problems)} stencils of the suite on the full {problems[0].interior[0]}x"
                  f"{problems[0].interior[1]} grid, {steps} steps each ({updates:.3e} updates, "
                  f"{dt:.1f} s)",
    }


KERNEL_SOURCES = ("paper_2305_07390_amd/csrc/tb2d_impl.hpp",
                  "paper_2305_07390_amd/csrc/device_common.hpp")
TRAFFIC_PROFILE = "profiles/tb2d_traffic_2d_suite_8192.md"
KERNEL_SOURCES_3D = ("paper_2305_07390_amd/csrc/tb3d_impl.hpp",
                     "paper_2305_07390_amd/csrc/tb3d_dev_impl.hpp",
                     "paper_2305_07390_amd/csrc/device_common.hpp")
TRAFFIC_PROFILE_3D = "profiles/tb3d_traffic_3d_suite_512.md"
KERNEL_SOURCES_BATCH = ("paper_2305_07390_amd/csrc/batch_impl.hpp",
                        "paper_2305_07390_amd/csrc/worklist.hpp",
                        "paper_2305_07390_amd/csrc/tb2d_impl.hpp",
                        "paper_2305_07390_amd/csrc/tb3d_impl.hpp",
                        "paper_2305_07390_amd/csrc/device_common.hpp")
TRAFFIC_PROFILE_BATCH = "profiles/batch_traffic_128_grids.md"


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_tag: str, profile=TRAFFIC_PROFILE, sources=KERNEL_SOURCES):
    """HBM bytes per launch of `kernel_tag` from a committed PMC summary, or
    None if the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, profile)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    src = None
    for line in text.splitlines():
        if line.startswith("kernel source hash"):
            src = line.rsplit(":", 1)[1].strip()
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 6 and cells[0] == kernel_tag and src == kernel_source_hash(sources):
            try:
                return int(float(cells[5]))
            except ValueError:
                return None
    return None


def calibration_copy(torch):
    """A 512 MiB device copy: the known-size kernel that scales the HBM
    counters (FETCH_SIZE, WRITE_SIZE) of the other dispatches."""
    a = torch.empty(512 << 18, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"probe: copy of {a.numel() * 4} bytes")
    del a, b


def probe3d():
    """Short program for 3D counter passes: the calibration copy, two passes of
    each 3D suite stencil (512^3, FP64 and FP32) at its planned depth, and one
    device-tiled run of each at its deepest compiled depth over 2 x depth
    steps."""
    import numpy as np
    import torch

    from paper_2305_07390_amd import stencil, workloads
    torch.cuda.set_device(0)
    calibration_copy(torch)
    for prob in workloads.suite_3d_problems(512, 200):
        for dt in (np.float64, np.float32):
            x = torch.from_numpy(prob.field(dt)).cuda()
            y = torch.empty_like(x)
            full = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, dt, prob.T)
            d = full.info["depth"]
            full.close()
            plan = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, dt, 2 * d)
            plan.execute(x, y)
            torch.cuda.synchronize()
            log(f"probe3d: {prob.spec.name} {np.dtype(dt).name} depth {d} passes {plan.info['passes']}")
            plan.close()
            dev = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, dt, 64, depth=64,
                               flags=stencil.STENCIL_FLAG_DEVICE_TILING)
            dd = dev.info["depth"]
            dev.close()
            dev = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, dt, 2 * dd, depth=dd,
                               flags=stencil.STENCIL_FLAG_DEVICE_TILING)
            if dev.info["scheme_name"] == "device_3d":
                dev.execute(x, y)
                torch.cuda.synchronize()
                log(f"probe3d: {prob.spec.name} {np.dtype(dt).name} device tiling depth {dd}")
            dev.close()
            del x, y
            torch.cuda.empty_cache()


def probe_batch():
    """The calibration copy, then one run of the 128-grid batch per dtype (for
    kernel traces and counter passes)."""
    import numpy as np
    import torch

    from paper_2305_07390_amd import stencil, workloads
    torch.cuda.set_device(0)
    calibration_copy(torch)
    probs = workloads.batch_problems()
    for dt in (np.float64, np.float32):
        xs = [torch.from_numpy(p.field(np.float64).astype(dt)).cuda() for p in probs]
        ys = [torch.empty_like(x) for x in xs]
        stencil.run_batch(probs, xs, ys)
        stencil.stencil_sync()
        log(f"probe batch: {np.dtype(dt).name} {len(probs)} grids")
        del xs, ys
        torch.cuda.empty_cache()


def probe():
    """Short program for PMC passes: a 512 MiB device copy (counter
    calibration) and two passes of each suite stencil at its planned depth."""
    import numpy as np
    import torch

    from paper_2305_07390_amd import stencil, workloads
    torch.cuda.set_device(0)
    calibration_copy(torch)
    for prob in workloads.suite_2d_problems(8192, 1000):
        x = torch.from_numpy(prob.field()).cuda()
        y = torch.empty_like(x)
        full = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, prob.T)
        d = full.info["depth"]
        full.close()
        plan = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, 2 * d)
        plan.execute(x, y)
        torch.cuda.synchronize()
        log(f"probe: {prob.spec.name} depth {d} passes {plan.info['passes']}")
        plan.close()
        del x, y
        torch.cuda.empty_cache()


def timed(torch, fn):
    """Run fn once on the current stream between two events; seconds."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3


def bench_3d(torch, np, stencil, workloads, B_gbs, n=512, T=200):
    """3D single-grid suite, FP64: per stencil, the planner's plan (overlapped
    tiles) and the best device-tiled plan (every depth, over the same T), one
    timed run each after a warm-up; each row carries the roofline record of its pass
    kernel (HBM or VALU bound, the per-launch time from events around the
    execution divided by its passes) and the model's prediction."""
    rows, total_t, total_u = [], 0.0, 0
    S = 8
    for prob in workloads.suite_3d_problems(n, T):
        x = torch.from_numpy(prob.field(np.float64)).cuda()
        y = torch.empty_like(x)
        plan = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, prob.T)
        plan.execute(x, y)
        t = timed(torch, lambda: plan.execute(x, y))
        info = plan.info
        t_eff = prob.T / info["passes"]
        per_launch = t / info["passes"]
        r_hbm = t_eff * HBM_PEAK_GBS / (2 * S)
        r_valu = FP64_VALU_TFLOPS * 1e3 / (2 * prob.spec.points)
        gcells = prob.updates / t / 1e9
        if r_hbm <= r_valu:
            roof = {"bound": "hbm", "achieved": round(2 * S * prob.cells / per_launch / 1e9, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        else:
            roof = {"bound": "alu", "achieved": round(2 * prob.spec.points * prob.cells * info["depth"]
                                                      / per_launch / 1e12, 2),
                    "peak": FP64_VALU_TFLOPS, "unit": "TFLOP/s"}
        roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
        tag = f"tb3d<double,{prob.spec.r},{info['pattern']},{info['depth']}>"
        roof["traffic"] = measured_traffic(tag, TRAFFIC_PROFILE_3D, KERNEL_SOURCES_3D)
        roof["kernel_source"] = kernel_source_hash(KERNEL_SOURCES_3D)
        row = {"stencil": prob.spec.name, "scheme": info["scheme_name"], "depth": info["depth"],
               "passes": info["passes"], "ms": round(t * 1e3, 2), "gcells_per_s": round(gcells, 1),
               "avg_launch_us": round(per_launch * 1e6, 2),
               "fraction": round(gcells / min(t_eff * B_gbs / (2 * S), r_valu), 4),
               "fraction_spec_hbm": round(gcells / min(r_hbm, r_valu), 4),
               "model_gcells_per_s": round(info["model_cells_per_s"] / 1e9, 1), "roofline": roof}
        plan.close()
        # device tiling: every compiled depth, over the same T steps (the
        # frame copies and the ring reset of a run amortised as above)
        best = None
        dmax = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, prob.T,
                            flags=stencil.STENCIL_FLAG_DEVICE_TILING).info
        if dmax["scheme_name"] == "device_3d":
            for d in range(1, dmax["depth"] + 1):
                Td = prob.T
                dp = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, Td, depth=d,
                                  flags=stencil.STENCIL_FLAG_DEVICE_TILING)
                dp.execute(x, y)
                td = timed(torch, lambda: dp.execute(x, y))
                g = prob.cells * Td / td / 1e9
                if best is None or g > best["gcells_per_s"]:
                    best = {"depth": d, "gcells_per_s": round(g, 1),
                            "model_gcells_per_s": round(dp.info["model_cells_per_s"] / 1e9, 1)}
                dp.close()
        row["device_tiling_best"] = best
        rows.append(row)
        total_t += t
        total_u += prob.updates
        log(f"  3d {rows[-1]}")
        del x, y
        torch.cuda.empty_cache()
    return {"workload": f"3D single-grid suite {n}^3 FP64, T={T}", "gcells_per_s":
            round(total_u / total_t / 1e9, 1), "per_stencil": rows}


def bench_persistent(torch, np, stencil, problems, xs, ys):
    """The 2D suite with every pass of a grid in one persistent launch
    (inter-pass synchronisation through the grid-wide tile count)."""
    rows, total_t, total_u = [], 0.0, 0
    for prob, x, y in zip(problems, xs, ys):
        plan = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, prob.T,
                            flags=stencil.STENCIL_FLAG_PERSISTENT)
        plan.execute(x, y)
        stencil.stencil_sync()
        t = timed(torch, lambda: plan.execute(x, y))
        stencil.stencil_sync()
        rows.append({"stencil": prob.spec.name, "depth": plan.info["depth"], "passes": plan.info["passes"],
                     "ms": round(t * 1e3, 2), "gcells_per_s": round(prob.updates / t / 1e9, 1)})
        total_t += t
        total_u += prob.updates
        log(f"  persistent {rows[-1]}")
        plan.close()
    return {"workload": "2D single-grid suite, all passes in one persistent launch per grid",
            "gcells_per_s": round(total_u / total_t / 1e9, 1), "per_stencil": rows}


def bench_autotune(torch, np, stencil, problems, xs, ys):
    """Autotuner on the 2D suite: tune each stencil at its full size (model-
    pruned candidates timed on the device), then time the plan the cache
    now picks for a plan without hints, next to the default plan."""
    stencil.stencil_tune_cache_clear()
    rows = []
    for prob, x, y in zip(problems, xs, ys):
        t0 = time.perf_counter()
        res = stencil.stencil_tune(prob.coeffs, prob.spec.r, prob.interior, np.float64)
        tune_s = time.perf_counter() - t0
        plan = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, prob.T)
        plan.execute(x, y)
        t = timed(torch, lambda: plan.execute(x, y))
        rows.append({"stencil": prob.spec.name, "depth": plan.info["depth"], "seg_len": plan.info["seg_len"],
                     "candidates": res["candidates"], "tune_s": round(tune_s, 2),
                     "gcells_per_s": round(prob.updates / t / 1e9, 1)})
        log(f"  tuned {rows[-1]}")
        plan.close()
    stencil.stencil_tune_cache_clear()
    return {"workload": "2D single-grid suite, plans from the autotuner's cache", "per_stencil": rows}


def bench_naive(torch, np, stencil, problems, xs, ys, T=20):
    """GCells/s of the plain one-step-per-launch kernel (t = 1) on the suite."""
    rows = []
    for prob, x, y in zip(problems, xs, ys):
        plan = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, T,
                            flags=stencil.STENCIL_FLAG_NAIVE)
        plan.execute(x, y)
        t = timed(torch, lambda: plan.execute(x, y))
        rows.append({"stencil": prob.spec.name, "T": T, "gcells_per_s": round(prob.cells * T / t / 1e9, 1)})
        plan.close()
    return rows


def bench_small_jacobi(torch, np, stencil, workloads, reps=20):
    """The small Jacobi workload (256^2 interior, T = 16, FP64): latency of one
    stencil_execute (launch-bound) and of stencil_run (planning included)."""
    prob = workloads.small_jacobi_problem()
    x = torch.from_numpy(prob.field(np.float64)).cuda()
    y = torch.empty_like(x)
    plan = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, prob.T)
    plan.execute(x, y)
    lat = sorted(timed(torch, lambda: plan.execute(x, y)) for _ in range(reps))
    stream = torch.cuda.current_stream().cuda_stream
    torch.cuda.synchronize()
    wall = []
    for _ in range(reps):
        t0 = time.perf_counter()
        stencil.stencil_run(prob.coeffs, prob.spec.r, prob.interior, np.float64, prob.T, x.data_ptr(),
                            y.data_ptr(), stream)
        torch.cuda.synchronize()
        wall.append(time.perf_counter() - t0)
    wall.sort()
    out = {"workload": "2D 5-point Jacobi, weights 0.2, 256x256 FP64 interior, T=16",
           "scheme": plan.info["scheme_name"], "depth": plan.info["depth"],
           "execute_us_median": round(lat[len(lat) // 2] * 1e6, 1), "execute_us_best": round(lat[0] * 1e6, 1),
           "run_wall_us_median": round(wall[len(wall) // 2] * 1e6, 1)}
    plan.close()
    return out


def batch_bound_seconds(np, stencil, probs, dtype, B):
    """max(sum of algorithmic bytes / B, sum of flops / F) for a batch: each
    pass of the plan the batch runs a job with reads and writes its grid once."""
    S = 8 if dtype == np.float64 else 4
    F = (FP64_VALU_TFLOPS if dtype == np.float64 else FP32_VALU_TFLOPS) * 1e12
    nbytes = 0.0
    nflops = 0.0
    for p in probs:
        info = stencil.stencil_batch_describe(p.coeffs, p.spec.r, p.interior, dtype, p.T)
        nbytes += 2.0 * S * p.cells * info["passes"]
        nflops += 2.0 * p.spec.points * p.updates
    return max(nbytes / (B * 1e9), nflops / F), nbytes, nflops


def bench_paper_benchmarks(torch, np, stencil, workloads):
    """The paper's nine benchmark stencils at its own domain sizes (FP64; the
    17- and 19-point 3D sets as defined in workloads), planner defaults."""
    rows = []
    for prob in workloads.paper_benchmark_problems():
        x = torch.from_numpy(prob.field(np.float64)).cuda()
        y = torch.empty_like(x)
        plan = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, prob.T)
        plan.execute(x, y)
        t = timed(torch, lambda: plan.execute(x, y))
        rows.append({"stencil": prob.spec.name, "points": prob.spec.points,
                     "domain": list(prob.interior[::-1]), "T": prob.T, "scheme": plan.info["scheme_name"],
                     "depth": plan.info["depth"], "gcells_per_s": round(prob.updates / t / 1e9, 1)})
        log(f"  paper {rows[-1]}")
        plan.close()
        del x, y
        torch.cuda.empty_cache()
    return {"workload": "the paper's benchmark stencils at its domain sizes (x fastest), FP64", "per_stencil": rows}


def bench_model_calibration(np, stencil, breakdown, B_gbs):
    """The attainable-performance model (paper Section 5) per suite stencil:
    the planner's own prediction for the plan it chose (the plan's computed
    cells, traffic and flops under the library's machine parameters, measured
    on MI355X), the same model at spec parameters (8 TB/s, 78.6 TF), and the
    measured rate."""
    rows = []
    spec = {"hbm_bytes_per_s": HBM_PEAK_GBS * 1e9, "fp64_flops": FP64_VALU_TFLOPS * 1e12,
            "fp32_flops": FP32_VALU_TFLOPS * 1e12}
    machine = stencil.stencil_machine_get()
    for row in breakdown:
        out = {"stencil": row["stencil"], "depth": row["depth"], "measured": row["gcells_per_s"],
               "model_machine": round(row["model_gcells_per_s"], 1)}
        out["measured_over_model_machine"] = round(row["gcells_per_s"] / max(row["model_gcells_per_s"], 1e-9), 3)
        rows.append(out)
    return {"note": "model_machine: stencil_plan_info.model_cells_per_s of the executed plan under the "
                    "library's machine parameters", "machine": machine, "spec_parameters": spec,
            "copy_probe_GBs": round(B_gbs, 1), "per_stencil": rows}


def bench_batch(torch, np, stencil, workloads):
    """128 heterogeneous grids, one batched submission per dtype."""
    probs = workloads.batch_problems()
    upd = sum(p.updates for p in probs)
    out = {"workload": "128 grids: 2D sides log-U[512,4096], 3D log-U[64,256], T~U{50..500}, "
                       "7 stencil types", "grids": len(probs), "cell_updates": upd}
    ys_by = {}
    for dt, name in ((np.float64, "f64"), (np.float32, "f32")):
        xs = [torch.from_numpy(p.field(np.float64).astype(dt)).cuda() for p in probs]
        ys = [torch.empty_like(x) for x in xs]
        stencil.run_batch(probs, xs, ys)
        stencil.stencil_sync()
        t = timed(torch, lambda: stencil.run_batch(probs, xs, ys))
        stencil.stencil_sync()
        bound, nbytes, nflops = batch_bound_seconds(np, stencil, probs, dt, bench_batch.B)
        out[name] = {"s": round(t, 4), "gcells_per_s": round(upd / t / 1e9, 1),
                     "bound_s": round(bound, 4), "fraction_of_bound": round(bound / t, 4),
                     "algorithmic_GB": round(nbytes / 1e9, 2), "tflop": round(nflops / 1e12, 2)}
        # HBM bytes per launch of each batch kernel from the committed counter
        # summary (None once the kernel sources changed)
        tname = "double" if dt == np.float64 else "float"
        kernels = (f"batch<{tname},0>", f"batch<{tname},1>") if dt == np.float64 else (f"batch<{tname},0>",)
        traffic = {k: measured_traffic(k, TRAFFIC_PROFILE_BATCH, KERNEL_SOURCES_BATCH) for k in kernels}
        out[name]["traffic_bytes"] = traffic
        if all(v is not None for v in traffic.values()):
            out[name]["traffic_over_algorithmic"] = round(sum(traffic.values()) / nbytes, 3)
        out[name]["kernel_source"] = kernel_source_hash(KERNEL_SOURCES_BATCH)
        log(f"  batch {name}: {out[name]}")
        ys_by[name] = ys
        del xs
    err = 0.0
    for a, b in zip(ys_by["f64"], ys_by["f32"]):
        scale = float(a.abs().max())
        err = max(err, float((b.double() - a).abs().max()) / max(scale, 1e-300))
    out["f32_max_err_rel_to_max"] = err
    del ys_by
    torch.cuda.empty_cache()
    return out


def bench_serving(np, torch, stencil, workloads, seconds=10.0, rate=200.0, warmup=200):
    """Serving loop under open-loop Poisson arrivals, FP32, 200 GB budget:
    `warmup` requests, then the measured ones (seconds * rate); latency from
    submit to the end of the round that completes the request (H2D included).
    Also: FP32 error against the FP64 path on a seeded 5% sample plus the 10
    largest requests, FP64 plain throughput (one plan at a time) on the first
    200 measured requests, and a stress run with a 0.5 GB budget at 2x rate."""
    from paper_2305_07390_amd import serving
    measured = max(1, int(seconds * rate))
    count = warmup + measured
    reqs, arr = workloads.serving_requests(count, rate_hz=rate, dtype=np.float32)
    span = float(arr[-1] - arr[warmup]) if measured > 1 else 1.0
    offered = sum(p.cells * T for p, _, T in reqs[warmup:]) / max(span, 1e-9)
    rng = np.random.default_rng(6)
    sizes = [p.cells * T for p, _, T in reqs]
    sample = set(int(k) for k in rng.choice(np.arange(warmup, count), size=max(1, measured // 20),
                                            replace=False))
    sample |= set(int(k) for k in np.argsort(sizes)[-10:])
    kept = {}

    def keep(k, res):
        if k in sample:
            kept[k] = res
    with serving.Server(hbm_budget_bytes=200 * 10**9, max_slots=SERVE_SLOTS) as srv:
        res = serving.serve_open_loop(srv, reqs, arr, on_result=keep)
    # latency from each request's scheduled arrival (the open-loop client's lag to the
    # submit call included) to the end of the round that completes it
    alat = res["arrival_latency_s"]
    lat = np.array(alat[warmup:]) if len(alat) > warmup else np.array(alat)
    slat_srv = np.array(res["latency_s"][warmup:]) if len(res["latency_s"]) > warmup else np.array(res["latency_s"])
    s = res["stats"]
    # FP32 error against the FP64 path (bit-identical to the oracle in the parity tests)
    err = 0.0
    for k, got in kept.items():
        prob, field, T = reqs[k]
        x = torch.from_numpy(field.astype(np.float64)).cuda()
        y = torch.empty_like(x)
        plan = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, T)
        plan.execute(x, y)
        torch.cuda.synchronize()
        ref = y.cpu().numpy()
        plan.close()
        err = max(err, float(np.max(np.abs(got.astype(np.float64) - ref))) / float(np.max(np.abs(ref))))
    # FP64 plain on the same requests, one plan at a time
    sub = reqs[warmup:warmup + 200]
    t64 = 0.0
    u64 = 0
    for prob, field, T in sub:
        x = torch.from_numpy(field.astype(np.float64)).cuda()
        y = torch.empty_like(x)
        plan = stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, T)
        plan.execute(x, y)
        t64 += timed(torch, lambda: plan.execute(x, y))
        u64 += prob.cells * T
        plan.close()
    # the same arrivals with two rounds in flight (the next round enqueued
    # shortly before the running one ends): latency under this load
    with serving.Server(hbm_budget_bytes=200 * 10**9, max_slots=SERVE_SLOTS, rounds_in_flight=2) as srv:
        res2 = serving.serve_open_loop(srv, reqs, arr)
    a2 = res2["arrival_latency_s"]
    lat2 = np.array(a2[warmup:]) if len(a2) > warmup else np.array(a2)
    s2 = res2["stats"]
    two_rounds = {"completed": s2["completed"], "rounds": s2["rounds"],
                  "throughput_gcells_per_s": round(s2["cell_updates"] / max(s2["wall_s"], 1e-9) / 1e9, 1),
                  "p50_ms": round(float(np.percentile(lat2, 50)) * 1e3, 2),
                  "p99_ms": round(float(np.percentile(lat2, 99)) * 1e3, 2),
                  "mean_ms": round(float(lat2.mean()) * 1e3, 2)}
    log(f"  serving, two rounds in flight: {two_rounds}")
    # saturation sweep: offered load past the served capacity; the served
    # throughput plateaus at the capacity while p99 grows with the queue
    sweep = []
    for k, srate in enumerate((400.0, 800.0, 1600.0)):
        n_s = int(srate * 1.0)
        wreqs, warr = workloads.serving_requests(n_s, rate_hz=srate, seed=20 + k, dtype=np.float32)
        with serving.Server(hbm_budget_bytes=200 * 10**9, max_slots=SERVE_SLOTS) as srv:
            wres = serving.serve_open_loop(srv, wreqs, warr)
        ws = wres["stats"]
        wl_ = np.array(wres["arrival_latency_s"])
        woff = sum(p.cells * T for p, _, T in wreqs) / max(float(warr[-1] - warr[0]), 1e-9)
        sweep.append({"rate": srate, "requests": n_s, "offered_gcells_per_s": round(woff / 1e9, 1),
                      "served_gcells_per_s": round(ws["cell_updates"] / max(ws["wall_s"], 1e-9) / 1e9, 1),
                      "p50_ms": round(float(np.percentile(wl_, 50)) * 1e3, 2),
                      "p99_ms": round(float(np.percentile(wl_, 99)) * 1e3, 2),
                      # the open-loop client's lateness in submitting: the host staging of
                      # the inputs bounds the load that reaches the server
                      "submit_lag_ms": round(float(wres["submit_lag_s"]) * 1e3, 1)})
        log(f"  serving sweep {sweep[-1]}")
    # stress: small budget, twice the rate, so admission binds
    sreqs, sarr = workloads.serving_requests(400, rate_hz=2 * rate, seed=9, dtype=np.float32)
    with serving.Server(hbm_budget_bytes=5 * 10**8, max_slots=64) as srv:
        sres = serving.serve_open_loop(srv, sreqs, sarr)
    ss = sres["stats"]
    slat = np.array(sres["arrival_latency_s"])
    out = {"workload": f"Poisson arrivals {rate:g} req/s, {warmup} warm-up + {measured} measured requests, "
                       "grids drawn like the batch (pool of 32), FP32, 200 GB HBM budget, "
                       f"{SERVE_SLOTS} slots",
           "requests": count, "completed": s["completed"], "rejected": len(res["rejected"]),
           "offered_gcells_per_s": round(offered / 1e9, 1),
           "throughput_gcells_per_s": round(s["cell_updates"] / max(s["wall_s"], 1e-9) / 1e9, 1),
           "throughput_req_per_s": round(s["completed"] / max(s["wall_s"], 1e-9), 1),
           "latency_from": "scheduled arrival",
           "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
           "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
           "mean_ms": round(float(lat.mean()) * 1e3, 2),
           "p50_ms_from_submit": round(float(np.percentile(slat_srv, 50)) * 1e3, 2),
           "p99_ms_from_submit": round(float(np.percentile(slat_srv, 99)) * 1e3, 2),
           "rounds": s["rounds"],
           "max_active": s["max_active"], "hbm_peak_GB": round(s["hbm_peak"] / 1e9, 2),
           "submit_lag_ms": round(float(res["submit_lag_s"]) * 1e3, 2),
           "f32_max_err_rel_to_max": err, "f32_err_sample": len(kept),
           "fp64_plain_gcells_per_s_first200": round(u64 / max(t64, 1e-9) / 1e9, 1),
           "two_rounds_in_flight": two_rounds,
           "saturation_sweep": sweep,
           "served_fp32_capacity_gcells_per_s": max(r["served_gcells_per_s"] for r in sweep),
           "stress": {"budget_GB": 0.5, "rate": 2 * rate, "requests": 400, "completed": ss["completed"],
                      "rejected": len(sres["rejected"]), "max_active": ss["max_active"],
                      "hbm_peak_GB": round(ss["hbm_peak"] / 1e9, 2),
                      "p50_ms": round(float(np.percentile(slat, 50)) * 1e3, 2),
                      "p99_ms": round(float(np.percentile(slat, 99)) * 1e3, 2)}}
    log(f"  serving: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--T", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 3D suite, batch and serving measurements")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--depth", type=int, default=0, help="force a temporal depth (0 = plan)")
    ap.add_argument("--probe", action="store_true",
                    help="run the short program used for PMC counter passes and exit")
    ap.add_argument("--probe3d", action="store_true",
                    help="run the short 3D program used for counter passes and exit")
    ap.add_argument("--probe-batch", action="store_true",
                    help="run the 128-grid batch once per dtype and exit")
    args = ap.parse_args()
    if args.probe:
        probe()
        return
    if args.probe3d:
        probe3d()
        return
    if args.probe_batch:
        probe_batch()
        return

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2305_07390_amd import stencil, workloads

    torch.cuda.set_device(0)
    problems = workloads.suite_2d_problems(args.n, args.T)
    log(f"bench: 2D suite {args.n}^2 T={args.T}, {len(problems)} stencils")
    fields, xs, ys, plans = [], [], [], []
    for prob in problems:
        u0 = prob.field(np.float64)
        fields.append(u0)
        x = torch.from_numpy(u0).cuda()
        xs.append(x)
        ys.append(torch.empty_like(x))
        plans.append(stencil.Plan(prob.coeffs, prob.spec.r, prob.interior, np.float64, prob.T,
                                  depth=args.depth))
        log(f"  {prob.spec.name}: {plans[-1].info}")
    torch.cuda.synchronize()

    B = copy_bandwidth_probe(stencil)
    B_torch = copy_bandwidth(torch)
    log(f"copy bandwidth {B:.0f} GB/s (library probe), {B_torch:.0f} GB/s (torch copy)")

    stream = torch.cuda.current_stream()

    def step(events=None):
        for j, (plan, x, y) in enumerate(zip(plans, xs, ys)):
            if events is not None:
                events[j][0].record(stream)
            plan.execute(x, y, stream)
            if events is not None:
                events[j][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    per = [[0.0, 0, []] for _ in problems]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in problems]
        step(ev)
        torch.cuda.synchronize()
        for j, (a, b) in enumerate(ev):
            per[j][0] += a.elapsed_time(b) * 1e-3
            per[j][1] += 1
            per[j][2].append(a.elapsed_time(b) * 1e-3)
        log(f"  step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    updates_per_step = sum(p.updates for p in problems)
    value = updates_per_step * args.steps / wall / 1e9
    S = 8
    breakdown = []
    dominant = None
    for prob, plan, (tsum, cnt, ts) in zip(problems, plans, per):
        t = tsum / cnt
        ts = sorted(ts)
        info = plan.info
        t_eff = prob.T / info["passes"]
        gcells = prob.updates / t / 1e9
        r_hbm = t_eff * B / (2 * S)
        r_hbm_spec = t_eff * HBM_PEAK_GBS / (2 * S)
        r_valu = FP64_VALU_TFLOPS * 1e3 / (2 * prob.spec.points)
        per_launch = t / info["passes"]
        bytes_per_launch = 2 * S * prob.cells
        row = {
            "stencil": prob.spec.name, "points": prob.spec.points, "depth": info["depth"],
            "pattern_code": info["pattern"], "radius": prob.spec.r,
            "passes": info["passes"], "t_eff": round(t_eff, 3), "scheme": info["scheme_name"],
            "tiles": info["tiles"], "seg_len": info["seg_len"], "ms": round(t * 1e3, 3),
            "gcells_per_s": round(gcells, 2),
            "gcells_best": round(prob.updates / ts[0] / 1e9, 2),
            "gcells_median": round(prob.updates / ts[len(ts) // 2] / 1e9, 2),
            "roofline_gcells": round(min(r_hbm, r_valu), 1),
            "fraction": round(gcells / min(r_hbm, r_valu), 4),
            "fraction_spec_hbm": round(gcells / min(r_hbm_spec, r_valu), 4),
            "avg_launch_us": round(per_launch * 1e6, 2),
            "achieved_GBs": round(bytes_per_launch / per_launch / 1e9, 1),
            "tflops": round(2 * prob.spec.points * prob.updates / t / 1e12, 2),
            "model_gcells_per_s": round(info["model_cells_per_s"] / 1e9, 1),
        }
        breakdown.append(row)
        if dominant is None or t > dominant[0]:
            dominant = (t, row, bytes_per_launch, per_launch)

    _, drow, dbytes, dlaunch = dominant
    dprob = problems[[r["stencil"] for r in breakdown].index(drow["stencil"])]
    dtag = f"tb2d<double,{drow['radius']},{drow['pattern_code']},{drow['depth']}>"
    traffic = measured_traffic(dtag)
    # the bound of the dominant kernel: HBM (one read and one write of every
    # cell per pass) or VALU (2k flops per cell-update, depth updates per pass)
    hbm_rate = drow["t_eff"] * HBM_PEAK_GBS / (2 * S)
    valu_rate = FP64_VALU_TFLOPS * 1e3 / (2 * drow["points"])
    if hbm_rate <= valu_rate:
        roof = {"bound": "hbm", "achieved": round(dbytes / dlaunch / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    else:
        flops = 2 * drow["points"] * dprob.cells * drow["depth"]
        roof = {"bound": "alu", "achieved": round(flops / dlaunch / 1e12, 2), "peak": FP64_VALU_TFLOPS,
                "unit": "TFLOP/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["traffic"] = traffic
    roof["kernel"] = f"tb2d ({drow['stencil']}, depth {drow['depth']})"
    roof["kernel_source"] = kernel_source_hash()
    result = {
        "metric": "GCells/s (cell-updates per second), 2D single-grid suite",
        "value": round(value, 2),
        "unit": "GCells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"2D single-grid suite: {args.n}x{args.n} FP64 interior, T={args.T}, "
                        "5pt star r1 + 9pt box r1 + 13pt star r3 + 25pt box r2, Dirichlet halo",
            "grid": [args.n, args.n], "T": args.T, "stencils": [p.spec.name for p in problems],
        },
        "roofline": roof,
        "copy_bandwidth_GBs": round(B, 1),
        "copy_bandwidth_torch_GBs": round(B_torch, 1),
        "per_stencil": breakdown,
    }
    if not args.no_extras:
        log("2D suite, plain t=1 kernel ...")
        naive = bench_naive(torch, np, stencil, problems, xs, ys)
        for row, nv in zip(breakdown, naive):
            row["naive_t1_gcells_per_s"] = nv["gcells_per_s"]
        log("grid sync probe ...")
        result["grid_sync_us"] = round(stencil.stencil_probe_grid_sync(2000) * 1e6, 3)
        log("2D suite, persistent launches ...")
        result["suite_2d_persistent"] = bench_persistent(torch, np, stencil, problems, xs, ys)
        log("2D suite, autotuned ...")
        result["suite_2d_autotuned"] = bench_autotune(torch, np, stencil, problems, xs, ys)
    del xs, ys
    torch.cuda.empty_cache()
    if not args.no_extras:
        log("model calibration ...")
        result["model_calibration"] = bench_model_calibration(np, stencil, breakdown, B)
        log("paper benchmarks ...")
        result["paper_benchmarks"] = bench_paper_benchmarks(torch, np, stencil, workloads)
        log("small Jacobi ...")
        result["small_jacobi"] = bench_small_jacobi(torch, np, stencil, workloads)
        log("3D suite ...")
        result["suite_3d"] = bench_3d(torch, np, stencil, workloads, B)
        log("batch ...")
        bench_batch.B = B
        result["batch"] = bench_batch(torch, np, stencil, workloads)
        log("serving ...")
        result["serving"] = bench_serving(np, torch, stencil, workloads, seconds=args.serve_seconds)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(problems, fields)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
