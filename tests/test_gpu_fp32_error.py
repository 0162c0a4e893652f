"""FP32 fast form: error of the FP32 GPU path against the FP64 oracle, per
stencil and per T, held to a bound derived from the arithmetic.

Every stencil here has non-negative weights summing to 1, so one step maps
max|U| to at most max|U| and does not amplify earlier errors. One FP32 step
rounds each coefficient once (relative error <= u) and each of its k fused
multiply-adds once (relative error <= u of a partial sum bounded by max|U|),
u = 2^-24. So after T steps |U32 - U64| <= T (k + 1) u max|U0|. The measured
error is printed per case (it grows roughly like sqrt(T), far below the bound)."""
import json

import numpy as np
import pytest

import oracle
from paper_2305_07390_amd import workloads as wl

from tests.gpu_util import gpu_sweep

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
TS = (1, 10, 100)
SHAPES = {2: (512, 640), 3: (64, 72, 80)}
# the step counts of the workloads: T = 1000 (2D suite), T = 200 (3D suite),
# up to 500 (batch and serving), on 1024^2 and 128^3 grids
LONG = {2: ((1024, 1024), (500, 1000)), 3: ((128, 128, 128), (200, 500))}


@pytest.mark.parametrize("spec", wl.ALL_STENCILS, ids=[s.name for s in wl.ALL_STENCILS])
def test_fp32_error_against_fp64_oracle(spec):
    coeffs = wl.coeffs_for(spec, 500 + spec.r)
    assert np.all(coeffs >= 0) and abs(coeffs.sum() - 1) < 1e-12
    k = int(np.count_nonzero(coeffs))
    shape = SHAPES[spec.ndim]
    u64 = wl.make_field(shape, spec.r, seed=91, dtype=np.float64)
    u32 = u64.astype(np.float32)
    # the FP32 run starts from the rounded field; the oracle from the same values
    u0 = u32.astype(np.float64)
    umax = float(np.max(np.abs(u0)))
    rows = []
    for T in TS:
        ref = oracle.sweep(coeffs, spec.r, u0, T)
        got = gpu_sweep(coeffs, spec.r, u32, T).astype(np.float64)
        err = float(np.max(np.abs(got - ref)))
        bound = T * (k + 1) * U32 * umax
        rows.append({"stencil": spec.name, "T": T, "max_abs_err": err, "rel_to_max": err / umax,
                     "bound": bound})
        assert err <= bound, rows[-1]
    print(json.dumps(rows), flush=True)


@pytest.mark.parametrize("spec", wl.ALL_STENCILS, ids=[s.name for s in wl.ALL_STENCILS])
def test_fp32_error_at_workload_T(spec):
    coeffs = wl.coeffs_for(spec, 500 + spec.r)
    k = int(np.count_nonzero(coeffs))
    shape, ts = LONG[spec.ndim]
    u32 = wl.make_field(shape, spec.r, seed=93, dtype=np.float32)
    u0 = u32.astype(np.float64)
    umax = float(np.max(np.abs(u0)))
    rows = []
    for T in ts:
        ref = oracle.sweep(coeffs, spec.r, u0, T)
        got = gpu_sweep(coeffs, spec.r, u32, T).astype(np.float64)
        err = float(np.max(np.abs(got - ref)))
        bound = T * (k + 1) * U32 * umax
        rows.append({"stencil": spec.name, "shape": list(shape), "T": T, "max_abs_err": err,
                     "rel_to_max": err / umax, "bound": bound})
        assert err <= bound, rows[-1]
    print(json.dumps(rows), flush=True)
