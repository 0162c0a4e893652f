"""Plant plausible mistakes in copies of the oracle (on the CPU) and check that the
pins in ``tests/pins.py`` catch every one of them."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from tests import pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "oracle.c")

# (name, original text, replacement); the first occurrence is replaced, which is in
# the tap parser or in the float64 sweep.
MUTANTS = [
    ("mirrored_offsets", "int p = rem % side - r;", "int p = r - rem % side;"),
    ("transposed_axes", "for (int d = ndim - 1; d >= 0; --d) {\n      int p", "for (int d = 0; d < ndim; ++d) {\n      int p"),
    ("interior_extent_stride", "stride *= pext[d];", "stride *= pext[d] - 2 * r;"),
    ("dropped_last_term", "for (int q = 0; q < k; ++q) {\n          const double w", "for (int q = 0; q + 1 < k; ++q) {\n          const double w"),
    ("shifted_weights", "const double w = taps[q].w;", "const double w = taps[(q + 1) % k].w;"),
    ("in_place_update", "double *src = out, *dst = work;", "double *src = out, *dst = out;"),
    ("last_row_skipped", "hi[e] = n[d] + r;", "hi[e] = n[d] + r - (e == 1);"),
    ("one_step_short", "for (int64_t s = 0; s < T; ++s) {", "for (int64_t s = 1; s < T; ++s) {"),
    ("halo_updated", "lo[e] = r;\n    hi[e] = n[d] + r;", "lo[e] = r > 0 ? r - (e == 2 && ext[2] > 0) : 0;\n    hi[e] = n[d] + r;"),
]


# Mistakes in the float32 twin: accumulating in double and rounding once,
# keeping the coefficients in double, or rounding the product and the sum
# separately. Each keeps every float64 pin green.
F32_MUTANTS = [
    ("f32_accumulate_in_double",
     "for (int64_t x = lo[2]; x < hi[2]; ++x) acc[x] = 0.0f;\n        for (int q = 0; q < k; ++q) {\n"
     "          const float w = wf[q];\n          const float *nb = src + row + offs[q];\n"
     "          for (int64_t x = lo[2]; x < hi[2]; ++x) acc[x] = fmaf(w, nb[x], acc[x]);\n        }",
     "for (int64_t x = lo[2]; x < hi[2]; ++x) {\n          double a = 0.0;\n"
     "          for (int q = 0; q < k; ++q) a = fma((double)wf[q], (double)src[row + offs[q] + x], a);\n"
     "          acc[x] = (float)a;\n        }"),
    ("f32_unrounded_coefficients", "acc[x] = fmaf(w, nb[x], acc[x]);",
     "acc[x] = (float)fma(taps[q].w, (double)nb[x], (double)acc[x]);"),
    ("f32_unfused", "acc[x] = fmaf(w, nb[x], acc[x]);", "acc[x] = w * nb[x] + acc[x];"),
]


def _build(tmp_path, name, old, new, symbol="oracle_sweep_f64"):
    text = open(SRC).read()
    assert old in text, name
    mutated = text.replace(old, new, 1)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O1", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(so), str(c), "-lm"], check=True)
    lib = ctypes.CDLL(str(so))
    fn = getattr(lib, symbol)
    fn.restype = ctypes.c_int
    f32 = symbol.endswith("f32")
    P = ctypes.POINTER(ctypes.c_float if f32 else ctypes.c_double)
    PD = ctypes.POINTER(ctypes.c_double)
    fn.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, PD, ctypes.c_int64,
                   P, P, P, ctypes.c_int]
    dt = np.float32 if f32 else np.float64

    def sweep(coeffs, r, u0, T):
        u0 = np.ascontiguousarray(u0, dtype=dt)
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        n = np.array([s - 2 * r for s in u0.shape], dtype=np.int64)
        # the halo mutant reads one cell before the array; give it a guard band
        buf = np.zeros(u0.size + 64, dtype=dt)
        inn = buf[32:32 + u0.size]
        inn[:] = u0.ravel()
        out = np.zeros(u0.size + 64, dtype=dt)
        work = np.zeros(u0.size + 64, dtype=dt)
        fn(u0.ndim, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), r,
           c.ctypes.data_as(PD), T, inn.ctypes.data_as(P),
           out[32:].ctypes.data_as(P), work[32:].ctypes.data_as(P), 1)
        return out[32:32 + u0.size].reshape(u0.shape).copy()

    return sweep


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    sweep = _build(tmp_path, name, old, new)
    caught = []
    for cname, check in pins.ALL_CHECKS:
        try:
            check(sweep)
        except AssertionError:
            caught.append(cname)
        except (ValueError, IndexError, ZeroDivisionError):
            caught.append(cname)
    assert caught, f"mutant {name} passed every pin"


@pytest.mark.parametrize("name,old,new", F32_MUTANTS, ids=[m[0] for m in F32_MUTANTS])
def test_f32_mutant_is_caught(tmp_path, name, old, new):
    # the replaced text must sit in the float32 twin (after the float64 sweep)
    text = open(SRC).read()
    assert text.find(old) > text.find("oracle_sweep_f32"), name
    sweep = _build(tmp_path, name, old, new, symbol="oracle_sweep_f32")
    caught = []
    for cname, check in pins.F32_CHECKS:
        try:
            check(sweep)
        except AssertionError:
            caught.append(cname)
    assert caught, f"mutant {name} passed every float32 pin"
