"""Breakdown of this design's optimisations on one MI355X (paper Section 7,
breakdown study, redone for the 2D 5-point and 3D 7-point Jacobi stencils,
FP64): each step adds one optimisation to the previous one and is placed on
the roofline (operational intensity of the algorithmic bytes, attainable
rate at the spec and at the measured copy bandwidth, measured rate).

    python -m paper_2305_07390_amd.ablation build   # variant libraries (host)
    python -m paper_2305_07390_amd.ablation run     # every step (GPU), JSON + table

The variants are the library with some kernel optimisations compiled out
(the STENCIL_ABL_* switches of csrc/tb2d_impl.hpp and csrc/tb3d_impl.hpp);
each step runs in a child process that loads its variant through
$STENCIL_LIBRARY. Paper steps without a switch here: LST (the 2D inner loop
has no synchronisation to make lazy; the 3D exchange keeps one barrier per
level) and RST (every level is held in registers; there is no shared-memory
queue to replace)."""
from __future__ import annotations

import json
import os
import subprocess
import sys

from . import build as _build

FP64_PEAK_TFLOPS = 78.6
HBM_SPEC_GBS = 8000.0

# variant -> switches; only the FP64 radius-1 kernels are recompiled
VARIANTS = {
    "base": {"STENCIL_ABL_PREFETCH": 0, "STENCIL_ABL_SCHED_BARRIER": 0, "STENCIL_ABL_SPLIT_BODY": 0,
             "STENCIL_ABL_XCD_ORDER": 0, "STENCIL_ABL_PLANES": 2},
    "pre": {"STENCIL_ABL_SCHED_BARRIER": 0, "STENCIL_ABL_SPLIT_BODY": 0, "STENCIL_ABL_XCD_ORDER": 0},
    "sched": {"STENCIL_ABL_SPLIT_BODY": 0, "STENCIL_ABL_XCD_ORDER": 0},
    "split": {"STENCIL_ABL_XCD_ORDER": 0},
}
ONLY = ["tb2d_f64_r1.hip", "tb3d_f64_r1.hip"]

# (step, what it adds, variant or None for the library, plan depth, plan flags)
NAIVE, UNIFORM, DEVICE, OVERLAPPED = 1, 8, 16, 32
STEPS = {
    "2d": [
        ("plain", "one plain step per launch (t = 1)", None, 1, NAIVE),
        ("BASE", "blocked pass at depth 1: register streaming, DPP neighbours, no prefetch, one tile "
                 "body, uniform segments", "base", 1, UNIFORM),
        ("+CMQ", "depth 12: one register queue per time level", "base", 12, UNIFORM),
        ("+PRE", "rows loaded three ahead into a register ring", "pre", 12, UNIFORM),
        ("+SCHED", "each row's prefetch kept at the head of its row", "sched", 12, UNIFORM),
        ("+SPLIT", "interior strips without halo reads", "split", 12, UNIFORM),
        ("+EDGE", "edge strips with their own, shorter segments", "split", 12, 0),
        ("+XCD", "consecutive tile groups per XCD (the library)", None, 12, 0),
    ],
    "3d": [
        ("plain", "one plain step per launch (t = 1)", None, 1, NAIVE),
        ("BASE", "device tiling at depth 1 (the paper's 3D BASE)", None, 1, DEVICE),
        ("+CMQ", "device tiling at depth 6: one queue per time level", None, 6, DEVICE),
        ("SM tiles", "overlapped tiles at depth 4 instead, two planes in flight", "base", 4, OVERLAPPED),
        ("+PRE", "four planes in flight (the library)", None, 4, OVERLAPPED),
    ],
}
PROBLEMS = {"2d": ((8192, 8192), 1000, 5), "3d": ((512, 512, 512), 200, 7)}


def variant_path(name):
    return os.path.join(_build.VARIANTS, name, "libstencil.so")


def build_all():
    for name, defs in VARIANTS.items():
        _build.build_variant(name, defs, ONLY)


def _step(dim: str, idx: int) -> dict:
    """Child: time one step (best of three runs after a warm-up)."""
    import numpy as np
    import torch

    from . import stencil, workloads
    torch.cuda.set_device(0)
    interior, T, points = PROBLEMS[dim]
    # the first stencil of the bench's suite, same grid and T
    prob = (workloads.suite_2d_problems(interior[0], T) if dim == "2d"
            else workloads.suite_3d_problems(interior[0], T))[0]
    spec = prob.spec
    assert spec.points == points and tuple(prob.interior) == interior
    x = torch.from_numpy(prob.field(np.float64)).cuda()
    y = torch.empty_like(x)
    name, _, _, depth, flags = STEPS[dim][idx]
    plan = stencil.Plan(prob.coeffs, spec.r, interior, np.float64, T, depth=depth,
                        flags=flags | stencil.STENCIL_FLAG_NO_CACHE)
    plan.execute(x, y)
    torch.cuda.synchronize()
    best = None
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.execute(x, y)
        e1.record()
        e1.synchronize()
        t = e0.elapsed_time(e1) * 1e-3
        best = t if best is None else min(best, t)
    info = plan.info
    import hashlib
    out = {"dim": dim, "step": name, "scheme": info["scheme_name"], "depth": info["depth"],
           "passes": info["passes"], "s": best, "gcells_per_s": prob.cells * T / best / 1e9,
           "digest": hashlib.sha1(y.cpu().numpy().tobytes()).hexdigest()[:16]}
    if idx == len(STEPS[dim]) - 1:
        out["copy_GBs"] = stencil.stencil_probe_copy(1 << 30) / 1e9
    plan.close()
    return out


def run():
    rows = []
    for dim in ("2d", "3d"):
        for idx, (name, what, variant, _, _) in enumerate(STEPS[dim]):
            env = dict(os.environ)
            if variant:
                env["STENCIL_LIBRARY"] = variant_path(variant)
                if not os.path.exists(env["STENCIL_LIBRARY"]):
                    raise SystemExit(f"{env['STENCIL_LIBRARY']} missing: run `ablation build` first")
            else:
                env.pop("STENCIL_LIBRARY", None)
            print(f"ablation: {dim} {name}", file=sys.stderr, flush=True)
            res = subprocess.run([sys.executable, "-m", "paper_2305_07390_amd.ablation", "step", dim, str(idx)],
                                 env=env, capture_output=True, text=True, timeout=600)
            if res.returncode != 0:
                raise SystemExit(f"step {dim} {name} failed:\n{res.stderr[-2000:]}")
            row = json.loads(res.stdout.strip().splitlines()[-1])
            row["adds"] = what
            rows.append(row)
            print(json.dumps(row), flush=True)
    # every step computes the same terms in the same order: identical outputs
    for dim in ("2d", "3d"):
        digests = {r["digest"] for r in rows if r["dim"] == dim}
        if len(digests) != 1:
            raise SystemExit(f"{dim}: the steps' outputs differ: {digests}")
    # roofline placement: algorithmic bytes 2 x 8 B per cell and pass, 2k flops per cell-update
    for dim in ("2d", "3d"):
        sel = [r for r in rows if r["dim"] == dim]
        B = sel[-1]["copy_GBs"]
        k = PROBLEMS[dim][2]
        T = PROBLEMS[dim][1]
        print(f"\n{dim.upper()} {PROBLEMS[dim][0]} FP64, T = {T}; copy bandwidth {B:.0f} GB/s")
        print("| step | adds | scheme, depth | GCells/s | OI (flop/B) | attainable at 8 TB/s | at copy BW | "
              "fraction of attainable (copy BW) |")
        print("|---|---|---|---|---|---|---|---|")
        for r in sel:
            t_eff = T / r["passes"]
            oi = 2 * k * t_eff / 16.0
            att_spec = min(t_eff * HBM_SPEC_GBS / 16.0, FP64_PEAK_TFLOPS * 1e3 / (2 * k))
            att_copy = min(t_eff * B / 16.0, FP64_PEAK_TFLOPS * 1e3 / (2 * k))
            print(f"| {r['step']} | {r['adds']} | {r['scheme']}, {r['depth']} | {r['gcells_per_s']:.0f} | "
                  f"{oi:.2f} | {att_spec:.0f} | {att_copy:.0f} | {r['gcells_per_s'] / att_copy:.2f} |")


if __name__ == "__main__":
    cmd = sys.argv[1] if len(sys.argv) > 1 else "run"
    if cmd == "build":
        build_all()
    elif cmd == "step":
        print(json.dumps(_step(sys.argv[2], int(sys.argv[3]))), flush=True)
    else:
        run()
