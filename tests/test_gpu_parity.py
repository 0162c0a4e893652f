"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: FP64 max relative error <= 1e-12 over the interior (relative error as in
the oracle readings: |g - o| / max(|o|, 1e-6 max|o|)), halo cells bit-identical,
`in` unchanged, repeated runs bit-identical. The kernels accumulate in the
oracle's order, so results are also expected to be bit-identical; that is
asserted separately."""
import numpy as np
import pytest

import oracle
from paper_2305_07390_amd import workloads as wl
from tests import pins
from tests.gpu_util import gpu_sweep, halo_mask, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _check(coeffs, r, u0, T, **kw):
    got, info = gpu_sweep(coeffs, r, u0, T, return_info=True, repeats=2, **kw)
    ref = oracle.sweep(coeffs, r, u0, T)
    m = halo_mask(u0.shape, r)
    assert np.array_equal(got[m], u0[m]), "halo changed"
    if u0.dtype == np.float64:
        err = rel_err(got, ref, r)
        assert err <= TOL64, (err, info)
    assert np.array_equal(got, ref), ("not bit-identical to the oracle", rel_err(got, ref, r), info)
    return info


# (name, ndim, kind, r, interior, T)
CASES_2D = [
    ("5pt_256sq_T16", "star", 1, (256, 256), 16),
    ("5pt_ragged_T1", "star", 1, (333, 517), 1),
    ("5pt_ragged_T9", "star", 1, (333, 517), 9),
    ("5pt_ragged_T10", "star", 1, (333, 517), 10),
    ("5pt_ragged_T11", "star", 1, (333, 517), 11),
    ("5pt_ragged_T37", "star", 1, (701, 1109), 37),
    ("9box_ragged_T13", "box", 1, (419, 700), 13),
    ("13star_r3_T9", "star", 3, (300, 901), 9),
    ("25box_r2_T7", "box", 2, (281, 640), 7),
    ("9star_r2_T11", "star", 2, (257, 611), 11),
    ("star_r4_T5", "star", 4, (200, 700), 5),
    ("box_r3_T4", "box", 3, (150, 520), 4),
    ("box_r4_T3", "box", 4, (99, 600), 3),
    ("5pt_tall_T21", "star", 1, (2000, 260), 21),
    ("5pt_short_T12", "star", 1, (3, 1000), 12),
    ("5pt_one_row_T5", "star", 1, (1, 700), 5),
]


@pytest.mark.parametrize("name,kind,r,interior,T", CASES_2D, ids=[c[0] for c in CASES_2D])
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_parity_2d(name, kind, r, interior, T, dtype):
    seed = abs(hash(name)) % 1000
    w = wl.random_coeffs(2, kind, r, seed)
    u0 = wl.make_field(interior, r, seed, dtype)
    _check(w, r, u0, T)


def test_config1_uniform_5pt():
    prob = wl.small_jacobi_problem()
    u0 = prob.field()
    info = _check(prob.coeffs, 1, u0, prob.T)
    assert info["scheme_name"] == "blocked_2d"


@pytest.mark.parametrize("depth", [1, 2, 5, 8, 12])
def test_depth_invariance(depth):
    w = wl.random_coeffs(2, "star", 1, 77)
    u0 = wl.make_field((400, 777), 1, 77)
    info = _check(w, 1, u0, 25, depth=depth)
    assert info["depth"] == depth


@pytest.mark.parametrize("seg", [16, 37, 100, 1000])
def test_segment_invariance(seg):
    w = wl.random_coeffs(2, "box", 1, 78)
    u0 = wl.make_field((450, 800), 1, 78)
    _check(w, 1, u0, 14, seg_len=seg, depth=7)


@pytest.mark.parametrize("kind,r,interior,T,seg,depth", [
    ("star", 1, (450, 1300), 26, 100, 12), ("box", 1, (611, 1333), 17, 150, 8),
    ("star", 3, (500, 1200), 9, 120, 4), ("box", 2, (403, 1000), 11, 90, 5),
    ("star", 2, (700, 1500), 8, 1000, 7)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_edge_strip_segments(kind, r, interior, T, seg, depth, dtype):
    """Edge strips with their own shorter segments give the oracle's result,
    the same bits as the uniform tiling (at depths deep enough for three or
    more strips, which the edge split needs)."""
    w = wl.random_coeffs(2, kind, r, 83)
    u0 = wl.make_field(interior, r, 83, dtype)
    info = _check(w, r, u0, T, seg_len=seg, depth=depth)
    assert info["edge_tiles"] > 0 and info["edge_seg_len"] < info["seg_len"], info
    got = gpu_sweep(w, r, u0, T, seg_len=seg, depth=depth, flags=8)
    ref = gpu_sweep(w, r, u0, T, seg_len=seg, depth=depth)
    assert np.array_equal(got, ref)


def test_general_pattern():
    w = wl.random_coeffs(2, "box", 1, 79)
    w[0, 2] = 0.0
    w[2, 1] = 0.0
    u0 = wl.make_field((300, 600), 1, 79)
    info = _check(w, 1, u0, 7)
    assert info["pattern_name"] == "general"


def test_naive_paths():
    w = wl.random_coeffs(2, "star", 1, 80)
    u0 = wl.make_field((50, 60), 1, 80)  # narrower than one wave tile: plain kernel
    info = _check(w, 1, u0, 6)
    assert info["scheme_name"] == "naive"
    info = _check(w, 1, wl.make_field((300, 600), 1, 81), 6, flags=1)
    assert info["scheme_name"] == "naive"


def test_r0_and_T0():
    u0 = wl.make_field((40, 300), 0, 82)
    _check(np.array([[0.9]]), 0, u0, 5)
    w = wl.random_coeffs(2, "star", 1, 83)
    u1 = wl.make_field((40, 300), 1, 83)
    got = gpu_sweep(w, 1, u1, 0)
    assert np.array_equal(got, u1)


def test_all_zero_box():
    # no points: every step sets the interior to the empty sum, +0.0; the halo stays
    for shape, r in (((40, 300), 1), ((9, 20, 70), 2)):
        w = np.zeros((2 * r + 1,) * len(shape))
        u0 = wl.make_field(shape, r, 86)
        info = _check(w, r, u0, 3)
        assert info["points"] == 0
        got = gpu_sweep(w, r, u0, 3)
        inner = tuple(slice(r, -r) for _ in shape)
        assert np.all(got[inner] == 0.0) and not np.any(np.signbit(got[inner]))


def test_3d_small_plain():
    for kind, r in (("star", 1), ("box", 1), ("star", 2)):
        w = wl.poisson_like_coeffs(3, kind, r, 84)
        u0 = wl.make_field((17, 23, 29), r, 84)
        _check(w, r, u0, 5)


def test_dyadic_exact_bitwise():
    # exact regime: m + q*T <= 53
    nbox, u0_int = pins.dyadic_case(2, "box", 1, 4, 5, 85, (300, 560))
    w = nbox.astype(np.float64) / 16.0
    u0 = u0_int.astype(np.float64)
    got = gpu_sweep(w, 1, u0, 12)
    ref = oracle.sweep(w, 1, u0, 12)
    assert np.array_equal(got, ref)
    # every value is a multiple of 2^-48 below 2^53 * 2^-48
    scaled = got * 2.0 ** 48
    assert np.array_equal(scaled, np.round(scaled))


def test_pins_hold_on_gpu():
    """The closed-form pins also hold for the HIP path (on grids wide enough to
    take the blocked scheme)."""
    def sweep(coeffs, r, u0, T):
        return gpu_sweep(coeffs, r, u0, T)
    pins.check_constant(sweep, 2, "box", 2, T=9)
    pins.check_linear(sweep, 2, "star", 3, T=4)
    pins.check_composition(sweep, 2, "star", 1, T1=7, T2=12)


def test_general_pattern_r3_plain_fallback():
    w = wl.random_coeffs(2, "box", 3, 86)
    w[1, 5] = 0.0
    u0 = wl.make_field((120, 600), 3, 86)
    info = _check(w, 3, u0, 3)
    assert info["scheme_name"] == "naive" and info["pattern_name"] == "general"


# (name, kind, r, interior (z, y, x), T)
CASES_3D = [
    ("7pt_ragged_T1", "star", 1, (21, 70, 97), 1),
    ("7pt_ragged_T2", "star", 1, (21, 70, 97), 2),
    ("7pt_ragged_T5", "star", 1, (33, 131, 70), 5),
    ("7pt_wide_T7", "star", 1, (17, 64, 200), 7),
    ("27box_ragged_T3", "box", 1, (25, 90, 66), 3),
    ("27box_T6", "box", 1, (19, 140, 77), 6),
    ("13star_r2_T4", "star", 2, (20, 80, 90), 4),
    ("7pt_thin_z_T4", "star", 1, (2, 70, 70), 4),
]


@pytest.mark.parametrize("name,kind,r,interior,T", CASES_3D, ids=[c[0] for c in CASES_3D])
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_parity_3d(name, kind, r, interior, T, dtype):
    seed = abs(hash(name)) % 1000
    w = wl.poisson_like_coeffs(3, kind, r, seed)
    u0 = wl.make_field(interior, r, seed, dtype)
    _check(w, r, u0, T)


@pytest.mark.parametrize("seg", [8, 13, 40])
def test_3d_segment_invariance(seg):
    w = wl.random_coeffs(3, "star", 1, 87)
    u0 = wl.make_field((45, 75, 80), 1, 87)
    info = _check(w, 1, u0, 5, seg_len=seg)
    assert info["scheme_name"] == "blocked_3d"


def test_3d_general_pattern():
    w = wl.random_coeffs(3, "box", 1, 88)
    w[0, 0, 0] = 0.0
    u0 = wl.make_field((12, 70, 70), 1, 88)
    info = _check(w, 1, u0, 3)
    assert info["pattern_name"] == "general"


@pytest.mark.parametrize("kind", ["p17", "p19"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_parity_paper_3d_point_sets(kind, dtype):
    """The paper's 17- and 19-point 3D benchmark stencils (general pattern path)."""
    w = wl.poisson_like_coeffs(3, kind, 1, 91)
    u0 = wl.make_field((37, 70, 90), 1, 91, dtype)
    info = _check(w, 1, u0, 5)
    assert info["scheme_name"] == "blocked_3d" and info["pattern_name"] == "general", info


@pytest.mark.parametrize("kind,r", [("star", 1), ("box", 1), ("star", 2), ("p19", 1)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_parity_3d_interior_tiles(kind, r, dtype):
    """Grids wide enough for tiles with redundant margins on all four sides,
    whose face values come from neighbouring tiles' stale data."""
    w = wl.poisson_like_coeffs(3, kind, r, 93)
    u0 = wl.make_field((14, 200, 300), r, 93, dtype)
    info = _check(w, r, u0, 9)
    assert info["scheme_name"] == "blocked_3d" and info["strips"] >= 16, info
