"""3D device tiling (paper Section 4.1): non-overlapping 64 x 16 tiles that
exchange their edges of every level through global memory after each z-step.
Bit-identical to the oracle for every supported stencil and dtype, at every
compiled depth, with full and remainder passes, odd and even pass counts,
single-tile and multi-tile grids (a 3 x 3 grid gives a tile with all eight
neighbours), grids barely deeper than the level pipeline, and at 512^3."""
import numpy as np
import pytest

import oracle
from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl
from tests.gpu_util import gpu_sweep

pytestmark = pytest.mark.gpu

DEV = st.STENCIL_FLAG_DEVICE_TILING


def _check(spec, interior, T, dtype=np.float64, depth=0, seed=3):
    coeffs = wl.coeffs_for(spec, seed)
    u0 = wl.make_field(interior, spec.r, seed + 1).astype(dtype)
    print(f"{spec.name} {interior} T={T} depth={depth} {np.dtype(dtype).name}", flush=True)
    got, info = gpu_sweep(coeffs, spec.r, u0, T, depth=depth, flags=DEV, repeats=2, return_info=True)
    assert info["scheme_name"] == "device_3d", info
    assert info["redundant_lanes"] == 0
    ref = oracle.sweep(coeffs, spec.r, u0, T)
    assert np.array_equal(got, ref), (spec.name, interior, T, depth, float(np.max(np.abs(got - ref))))
    return info


STAR1, BOX1, STAR2 = wl.SUITE_3D[0], wl.SUITE_3D[1], wl.SUITE_3D[2]


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("spec", [STAR1, BOX1, STAR2], ids=lambda s: s.name)
@pytest.mark.parametrize("interior", [(12, 32, 128), (20, 48, 192), (7, 16, 64), (9, 16, 256)],
                         ids=["2x2", "3x3", "1x1", "4x1"])
def test_parity_default_depth(spec, interior, dtype):
    # T = 2 d + 1: two full passes and a one-level remainder pass
    d = st.Plan(wl.coeffs_for(spec, 3), spec.r, interior, dtype, 1000, flags=DEV).info["depth"]
    _check(spec, interior, 2 * d + 1, dtype)


@pytest.mark.parametrize("spec", [STAR1, BOX1, STAR2], ids=lambda s: s.name)
def test_every_depth(spec):
    dmax = st.Plan(wl.coeffs_for(spec, 3), spec.r, (10, 32, 128), np.float64, 1000, flags=DEV).info["depth"]
    for depth in range(1, dmax + 1):
        info = _check(spec, (10, 32, 128), depth + 2, depth=depth)
        assert info["depth"] == depth


def test_short_grid_and_many_passes():
    # fewer planes than the level pipeline is deep; 11 passes
    _check(STAR1, (3, 32, 128), 85)
    _check(STAR2, (5, 16, 128), 23, np.float32)


def test_512_cube_fp64():
    d = st.Plan(wl.coeffs_for(STAR1, 3), 1, (512, 512, 512), np.float64, 1000, flags=DEV).info["depth"]
    info = _check(STAR1, (512, 512, 512), 2 * d + 1)
    assert info["strips"] == 256 and info["passes"] == 3
