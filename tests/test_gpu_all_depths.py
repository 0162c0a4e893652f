"""Every compiled depth of every blocked variant, bitwise against the oracle:
2D star / box / general at radius 1-4 and 3D overlapped tiles at radius 1-2,
FP64 and FP32, each run for T = 2d + 1 steps (two full passes and a
one-step remainder) on a ragged grid that spans several strips or tiles."""
import numpy as np
import pytest

from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl

from tests.test_gpu_parity import _check

pytestmark = pytest.mark.gpu

VARIANTS_2D = [("star", 1), ("star", 2), ("star", 3), ("star", 4), ("box", 1), ("box", 2), ("box", 3),
               ("box", 4), ("general", 1), ("general", 2)]
VARIANTS_3D = [("star", 1), ("star", 2), ("box", 1), ("box", 2), ("general", 1), ("general", 2)]
DTYPES = [np.float64, np.float32]


def _coeffs(ndim, kind, r, seed, poisson=False):
    # a general pattern: a box with one corner point absent (neither star nor box)
    base = "box" if kind == "general" else kind
    w = (wl.poisson_like_coeffs(ndim, base, r, seed) if poisson else wl.random_coeffs(ndim, base, r, seed)).copy()
    if kind == "general":
        w[(0,) * ndim] = 0.0
    return w


def _deepest(coeffs, r, interior, dtype, flags=0):
    p = st.Plan(coeffs, r, interior, dtype, 99, depth=99, flags=flags | st.STENCIL_FLAG_NO_CACHE)
    info = p.info
    p.close()
    return info


@pytest.mark.parametrize("kind,r", VARIANTS_2D, ids=[f"{k}_r{r}" for k, r in VARIANTS_2D])
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_every_2d_depth(kind, r, dtype):
    interior = (150, 1100)
    w = _coeffs(2, kind, r, 300 + r)
    u0 = wl.make_field(interior, r, 300 + r, dtype)
    top = _deepest(w, r, interior, dtype)
    assert top["scheme_name"] == "blocked_2d" and top["pattern_name"] == kind
    for d in range(1, top["depth"] + 1):
        info = _check(w, r, u0, 2 * d + 1, depth=d)
        assert info["depth"] == d and info["passes"] == 3


@pytest.mark.parametrize("kind,r", VARIANTS_3D, ids=[f"{k}_r{r}" for k, r in VARIANTS_3D])
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_every_3d_overlapped_depth(kind, r, dtype):
    interior = (13, 70, 140)
    w = _coeffs(3, kind, r, 310 + r, poisson=True)
    u0 = wl.make_field(interior, r, 310 + r, dtype)
    top = _deepest(w, r, interior, dtype, flags=st.STENCIL_FLAG_OVERLAPPED_TILING)
    if top["scheme_name"] == "naive":
        # radius-2 boxes and general patterns have no FP32 3D blocked kernel
        assert dtype == np.float32 and r == 2 and kind in ("box", "general")
        pytest.skip("no FP32 3D blocked kernel for this variant")
    assert top["scheme_name"] == "blocked_3d" and top["pattern_name"] == kind
    for d in range(1, top["depth"] + 1):
        info = _check(w, r, u0, 2 * d + 1, depth=d, flags=st.STENCIL_FLAG_OVERLAPPED_TILING)
        assert info["depth"] == d
