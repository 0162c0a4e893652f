"""One persistent launch for all passes of a grid (inter-pass grid
synchronisation through the count of finished tiles): the same result as the
pass-per-launch schedule and the oracle, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl
from tests.gpu_util import gpu_sweep

pytestmark = pytest.mark.gpu

CASES = [
    ("2d5pt_star_r1", (300, 700), 40, np.float64),
    ("2d25pt_box_r2", (257, 1100), 23, np.float32),
    ("2d13pt_star_r3", (512, 512), 17, np.float64),
    ("3d7pt_star_r1", (40, 70, 130), 9, np.float64),
    ("3d13pt_star_r2", (33, 64, 100), 7, np.float32),
    ("3d13pt_star_r2", (30, 70, 96), 5, np.float64),
    ("3d27pt_box_r1", (26, 70, 90), 5, np.float64),
    ("2d9pt_box_r1", (300, 1100), 19, np.float32),
]


@pytest.mark.parametrize("name,interior,T,dtype", CASES, ids=[c[0] + "_" + np.dtype(c[3]).name for c in CASES])
def test_persistent_equals_oracle(name, interior, T, dtype):
    spec = {s.name: s for s in wl.ALL_STENCILS}[name]
    coeffs = wl.coeffs_for(spec, 61)
    u0 = wl.make_field(interior, spec.r, seed=62, dtype=dtype)
    ref = oracle.sweep(coeffs, spec.r, u0, T)
    got, info = gpu_sweep(coeffs, spec.r, u0, T, flags=st.STENCIL_FLAG_PERSISTENT, repeats=2,
                          return_info=True)
    assert info["passes"] >= 2, info
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_persistent_edge_segments(dtype):
    """The persistent kernel follows a plan whose edge strips have their own segments."""
    spec = {s.name: s for s in wl.ALL_STENCILS}["2d9pt_box_r1"]
    coeffs = wl.coeffs_for(spec, 63)
    u0 = wl.make_field((450, 1300), 1, seed=64, dtype=dtype)
    ref = oracle.sweep(coeffs, 1, u0, 30)
    got, info = gpu_sweep(coeffs, 1, u0, 30, seg_len=100, flags=st.STENCIL_FLAG_PERSISTENT, repeats=2,
                          return_info=True)
    assert info["edge_tiles"] > 0 and info["passes"] >= 2, info
    np.testing.assert_array_equal(got, ref)


def test_grid_sync_probe():
    """One grid-wide barrier of one workgroup per CU costs microseconds, not
    milliseconds, and the probe leaves no device error behind."""
    t = st.stencil_probe_grid_sync(500)
    assert 0 < t < 1e-4, t
    st.stencil_sync()
    with pytest.raises(st.StencilError):
        st.stencil_probe_grid_sync(0)


@pytest.mark.parametrize("T", [1, 3, 12])
def test_persistent_single_pass_and_remainder(T):
    """A persistent plan whose passes are one short pass, or one full pass."""
    spec = {s.name: s for s in wl.ALL_STENCILS}["2d5pt_star_r1"]
    coeffs = wl.coeffs_for(spec, 65)
    u0 = wl.make_field((260, 900), 1, seed=66)
    ref = oracle.sweep(coeffs, 1, u0, T)
    got, info = gpu_sweep(coeffs, 1, u0, T, flags=st.STENCIL_FLAG_PERSISTENT, repeats=2, return_info=True)
    assert info["passes"] == 1, info
    np.testing.assert_array_equal(got, ref)
