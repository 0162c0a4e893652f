"""Build ``libstencil.so`` (HIP kernels for gfx950 + the C ABI) in-tree.

Every translation unit under ``csrc/`` is compiled with hipcc in parallel into
``_build/`` and linked into ``paper_2305_07390_amd/libstencil.so``. Run as
``python -m paper_2305_07390_amd.build`` or through ``__graft_entry__.build()``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libstencil.so")
ROOT = os.path.dirname(HERE)

ARCH = "gfx950"
# Packed FP32 instructions are kept out of every kernel: the compiler is told
# not to form them.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-I", CSRC, "-I", os.path.join(ROOT, "include")]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))


RESOURCE_REPORT = os.path.join(BUILD, "kernel_resources.txt")
_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]):\s*(\S+)")


def _resources(stderr: str):
    """Per-kernel register, scratch and LDS use from the compiler's resource
    remarks: [(name, {field: value})]."""
    out, cur = [], None
    for field, value in _REMARK.findall(stderr):
        if field == "Function Name":
            cur = (value, {})
            out.append(cur)
        elif cur is not None:
            cur[1][field.split(" ")[0]] = value
    return out


def _compile(src: str):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [_hipcc(), *COMMON, *DEVICE_FLAGS, "-Rpass-analysis=kernel-resource-usage", "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj, _resources(res.stderr)


def build(jobs: int | None = None, verbose: bool = True, only: list | None = None) -> str:
    """Compile every source (or, with `only`, just the named ones, reusing the
    other objects of the previous build) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    todo = [s for s in srcs if not only or os.path.basename(s) in only]
    jobs = jobs or max(1, min(len(todo), len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        done = dict(zip(todo, ex.map(_compile, todo)))
    objs = [done[s][0] if s in done else os.path.join(BUILD, os.path.basename(s) + ".o") for s in srcs]
    # one line per kernel: name, VGPRs, AGPRs, scratch bytes per lane, LDS
    old = {}
    if only and os.path.exists(RESOURCE_REPORT):
        for line in open(RESOURCE_REPORT):
            old.setdefault(line.split(" ", 1)[0], []).append(line)
    with open(RESOURCE_REPORT, "w") as f:
        for src in srcs:
            base = os.path.basename(src)
            if src not in done:
                f.writelines(old.get(base, []))
                continue
            for name, r in done[src][1]:
                f.write(f"{base} {name} vgpr={r.get('VGPRs')} agpr={r.get('AGPRs')} "
                        f"scratch={r.get('ScratchSize')} lds={r.get('LDS')}\n")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources", file=sys.stderr)
    return LIB


# Ablation variants (paper Section 7, breakdown study): the library with
# some kernel optimisations compiled out (the STENCIL_ABL_* switches of
# tb2d_impl.hpp and tb3d_impl.hpp). Only the named sources are recompiled;
# every other object comes from the default build, which must exist.
VARIANTS = os.path.join(HERE, "ablation_builds")


def build_variant(name: str, defines: dict, only: list, verbose: bool = True) -> str:
    objdir = os.path.join(BUILD, "abl_" + name)
    os.makedirs(objdir, exist_ok=True)
    outdir = os.path.join(VARIANTS, name)
    os.makedirs(outdir, exist_ok=True)
    flags = [f"-D{k}={v}" for k, v in sorted(defines.items())]
    objs = []
    for src in sources():
        base = os.path.basename(src)
        if base in only:
            obj = os.path.join(objdir, base + ".o")
            cmd = [_hipcc(), *COMMON, *DEVICE_FLAGS, *flags, "-Rpass-analysis=kernel-resource-usage", "-c", src,
                   "-o", obj]
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
            spills = [n for n, r in _resources(res.stderr) if r.get("ScratchSize") not in ("0", None)]
            if spills:
                raise RuntimeError(f"variant {name}: kernels spill to scratch: {spills}")
        else:
            obj = os.path.join(BUILD, base + ".o")
            if not os.path.exists(obj):
                raise RuntimeError(f"{obj} missing: build the library first")
        objs.append(obj)
    lib = os.path.join(outdir, "libstencil.so")
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", lib, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    if verbose:
        print(f"built {lib} ({', '.join(flags)})", file=sys.stderr)
    return lib


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="", help="comma-separated sources to recompile")
    a = ap.parse_args()
    build(only=[x for x in a.only.split(",") if x] or None)
