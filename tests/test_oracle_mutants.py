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


def _build(tmp_path, name, old, new):
    text = open(SRC).read()
    assert old in text, name
    mutated = text.replace(old, new, 1)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O1", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(so), str(c), "-lm"], check=True)
    lib = ctypes.CDLL(str(so))
    fn = lib.oracle_sweep_f64
    fn.restype = ctypes.c_int
    P = ctypes.POINTER(ctypes.c_double)
    fn.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, P, ctypes.c_int64,
                   P, P, P, ctypes.c_int]

    def sweep(coeffs, r, u0, T):
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        n = np.array([s - 2 * r for s in u0.shape], dtype=np.int64)
        # the halo mutant reads one cell before the array; give it a guard band
        buf = np.zeros(u0.size + 64)
        inn = buf[32:32 + u0.size]
        inn[:] = u0.ravel()
        out = np.zeros(u0.size + 64)
        work = np.zeros(u0.size + 64)
        fn(u0.ndim, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), r,
           c.ctypes.data_as(P), T, inn.ctypes.data_as(P),
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
