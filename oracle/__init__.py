"""CPU oracle for iterated out-of-place Jacobi stencil sweeps.

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product path
(``paper_2305_07390_amd``) never imports it, and the two share no code.

Contents:

* ``sweep`` -- the plain definition (paper Section 2.1, Listings 1-3), run by a
  small C library (``oracle.c``) with one full sweep per step, canonical
  summation order and a Dirichlet halo of width r held at its initial values.
* ``brute`` -- independent pure-Python checkers used to pin ``sweep``:
  memoised single-point recursion, exact dyadic arithmetic on integers, and
  closed forms (see ``brute.py``).

Every function here is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def _host_has_fma() -> bool:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("flags"):
                    return " fma " in (line.rstrip() + " ")
    except OSError:
        pass
    return False


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (plain C, OpenMP, no FP contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC"]
    if _host_has_fma():
        cmd.append("-mfma")  # inline the fused multiply-add; results are identical
    cmd += ["-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        for name, ptr in (("oracle_sweep_f64", ctypes.c_double), ("oracle_sweep_f32", ctypes.c_float)):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                           ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                           ctypes.POINTER(ptr), ctypes.POINTER(ptr), ctypes.POINTER(ptr),
                           ctypes.c_int]
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def sweep(coeffs: np.ndarray, r: int, u0: np.ndarray, T: int, threads: int | None = None) -> np.ndarray:
    """Return U^T for the padded initial field ``u0`` (halo included).

    ``coeffs`` is the dense (2r+1)^ndim float64 box (slowest offset first);
    exact zeros are absent points. ``u0`` has shape ``n_j + 2r`` per axis and
    dtype float64 or float32; the result has the same shape and dtype. The
    float32 path rounds the coefficients to float once and uses ``fmaf``.
    """
    lib = _load()
    u0 = np.ascontiguousarray(u0)
    ndim = u0.ndim
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    if c.shape != (2 * r + 1,) * ndim:
        raise ValueError("coeffs must have shape (2r+1,)*ndim")
    n = np.array([s - 2 * r for s in u0.shape], dtype=np.int64)
    if np.any(n < 1):
        raise ValueError("interior extents must be >= 1")
    out = np.empty_like(u0)
    work = np.empty_like(u0)
    nthr = default_threads() if threads is None else int(threads)
    if u0.dtype == np.float64:
        fn, ptr = lib.oracle_sweep_f64, ctypes.c_double
    elif u0.dtype == np.float32:
        fn, ptr = lib.oracle_sweep_f32, ctypes.c_float
    else:
        raise TypeError("u0 must be float32 or float64")
    rc = fn(ndim, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(r),
            c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(T),
            u0.ctypes.data_as(ctypes.POINTER(ptr)), out.ctypes.data_as(ctypes.POINTER(ptr)),
            work.ctypes.data_as(ctypes.POINTER(ptr)), nthr)
    if rc != 0:
        raise ValueError("oracle rejected arguments")
    return out
