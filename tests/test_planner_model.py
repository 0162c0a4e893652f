"""The model-driven planner (paper Sections 5-6) on the host: with the MI355X
machine parameters it picks, for every benchmark configuration, the scheme and
depth that measure fastest; the choice follows the parameters (a cheaper
neighbour synchronisation with plentiful bandwidth makes device tiling win in
3D; the compute-to-bandwidth ratio sets the depth); explicit scheme flags and
hints override it. No kernel runs."""
import numpy as np
import pytest

from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl

NC = st.STENCIL_FLAG_NO_CACHE


@pytest.fixture(autouse=True)
def default_machine():
    try:
        st.load_library()
    except st.StencilLibraryMissing:
        pytest.skip("libstencil.so not built")
    st.stencil_machine_set(None)
    yield
    st.stencil_machine_set(None)


def _plan(spec, interior, dtype, T, seed=2, **kw):
    p = st.Plan(wl.coeffs_for(spec, seed), spec.r, interior, dtype, T, flags=NC | kw.pop("flags", 0), **kw)
    info = p.info
    p.close()
    return info


def test_machine_defaults_are_the_measured_mi355x_values():
    m = st.stencil_machine_get()
    assert m["hbm_bytes_per_s"] == pytest.approx(5.1e12)
    assert m["lds_bytes_per_s"] == pytest.approx(68.7e12)
    assert m["fp64_flops"] == pytest.approx(256 * 4 * 16 * 2 * 2.15e9)
    assert m["fp32_flops"] == m["fp64_flops"]  # packed FP32 is not used
    assert m["grid_sync_s"] == pytest.approx(9.5e-6)
    assert m["neighbor_sync_s"] == pytest.approx(3.3e-6)
    assert m["cus"] == 256


def test_machine_set_validates_and_resets():
    with pytest.raises(st.StencilError):
        st.stencil_machine_set(hbm_bytes_per_s=0.0)
    st.stencil_machine_set(hbm_bytes_per_s=1e12)
    assert st.stencil_machine_get()["hbm_bytes_per_s"] == 1e12
    st.stencil_machine_set(None)
    assert st.stencil_machine_get()["hbm_bytes_per_s"] == pytest.approx(5.1e12)


# (workload, stencil index, expected scheme, expected depth); the depths are
# the fastest measured on the MI355X for these sizes
SUITE_2D_PICKS = [(0, 12), (1, 10), (2, 5), (3, 6)]
SUITE_3D_PICKS = [(0, 4), (1, 2), (2, 2)]


@pytest.mark.parametrize("idx,depth", SUITE_2D_PICKS, ids=[s.name for s in wl.SUITE_2D])
def test_2d_suite_8192_fp64(idx, depth):
    info = _plan(wl.SUITE_2D[idx], (8192, 8192), np.float64, 1000)
    assert info["scheme_name"] == "blocked_2d" and info["depth"] == depth
    assert info["model_cells_per_s"] > 0


@pytest.mark.parametrize("idx,depth", SUITE_3D_PICKS, ids=[s.name for s in wl.SUITE_3D])
def test_3d_suite_512_fp64_prefers_overlapped_tiles(idx, depth):
    spec = wl.SUITE_3D[idx]
    info = _plan(spec, (512, 512, 512), np.float64, 200, seed=3)
    assert info["scheme_name"] == "blocked_3d" and info["depth"] == depth
    # device tiling applies at 512^3 but the model predicts it slower: one
    # neighbour synchronisation per z-step against a sub-microsecond step
    dev = _plan(spec, (512, 512, 512), np.float64, 200, seed=3, flags=st.STENCIL_FLAG_DEVICE_TILING)
    assert dev["scheme_name"] == "device_3d"
    assert dev["model_cells_per_s"] < info["model_cells_per_s"]


def test_small_jacobi_workload():
    prob = wl.small_jacobi_problem()
    p = st.Plan(prob.coeffs, 1, prob.interior, np.float64, prob.T, flags=NC)
    assert p.info["scheme_name"] == "blocked_2d" and p.info["depth"] == 12 and p.info["passes"] == 2
    p.close()


def test_scheme_choice_follows_the_machine():
    # With plentiful HBM bandwidth the 3D pass is compute-bound: overlapped
    # tiles then pay for their redundant margins, device tiling does not, and
    # with a free neighbour synchronisation device tiling wins. With the
    # measured synchronisation cost the overlapped tiles win again. (At the
    # measured bandwidth the 64 x 16 device tile's edge traffic, a third of
    # its 160 edge cells per 1024 per level, keeps it behind either way: its
    # short side is below the minimum device tile of paper Section 6.4.)
    spec = wl.SUITE_3D[0]
    st.stencil_machine_set(neighbor_sync_s=0.0, hbm_bytes_per_s=100 * 5.1e12)
    info = _plan(spec, (512, 512, 512), np.float64, 200, seed=3)
    assert info["scheme_name"] == "device_3d"
    assert info["redundant_lanes"] == 0
    st.stencil_machine_set(None)
    st.stencil_machine_set(hbm_bytes_per_s=100 * 5.1e12)
    assert _plan(spec, (512, 512, 512), np.float64, 200, seed=3)["scheme_name"] == "blocked_3d"
    st.stencil_machine_set(None)
    m = st.stencil_model_eval(B_gm=5.1e12, B_sm=68.7e12, thr_cmp=1.0, cell_bytes=8, a_gm=2, a_sm=4, a_cmp=14,
                              D_gm=1, D_sm=1, D_cmp=1, D_all=1, t=1, rad=1,
                              tiling=2, tile=(64, 16))  # device tiling
    assert 16 < m["min_tile"] < 64


def test_scheme_flags_override_the_model():
    spec = wl.SUITE_3D[0]
    st.stencil_machine_set(neighbor_sync_s=0.0, hbm_bytes_per_s=100 * 5.1e12)
    info = _plan(spec, (512, 512, 512), np.float64, 200, seed=3, flags=st.STENCIL_FLAG_OVERLAPPED_TILING)
    assert info["scheme_name"] == "blocked_3d"
    st.stencil_machine_set(None)
    info = _plan(spec, (512, 512, 512), np.float64, 200, seed=3, flags=st.STENCIL_FLAG_DEVICE_TILING)
    assert info["scheme_name"] == "device_3d"
    # device tiling does not apply (x not a multiple of 64): overlapped tiles
    info = _plan(spec, (64, 64, 100), np.float64, 200, seed=3, flags=st.STENCIL_FLAG_DEVICE_TILING)
    assert info["scheme_name"] == "blocked_3d"


def test_desired_depth_follows_the_bandwidth_to_compute_ratio():
    # paper Section 6.2: the depth that moves the bound off global memory.
    # With ten times the compute throughput the 25-point box is HBM-bound at
    # every compiled depth and the deepest wins; with a tenth the redundant
    # margin's flops dominate and the shallowest wins.
    spec = wl.SUITE_2D[3]
    m = st.stencil_machine_get()
    st.stencil_machine_set(fp64_flops=10 * m["fp64_flops"])
    deep = _plan(spec, (8192, 8192), np.float64, 1000)["depth"]
    st.stencil_machine_set(fp64_flops=m["fp64_flops"] / 10)
    shallow = _plan(spec, (8192, 8192), np.float64, 1000)["depth"]
    assert deep == st.Plan(wl.coeffs_for(spec, 2), 2, (8192, 8192), np.float64, 1000, depth=64,
                           flags=NC).info["depth"]
    assert shallow < deep


def test_model_rate_counts_the_redundant_margin():
    # at equal depth, a wider 2D tile (FP32: 8 columns per lane) loses a
    # smaller share to its margins than the FP64 tile, so its predicted rate
    # is more than the 2x of halved bytes would give on HBM alone at depth 1
    spec = wl.SUITE_2D[0]
    f64 = _plan(spec, (8192, 8192), np.float64, 1000, depth=4)
    f32 = _plan(spec, (8192, 8192), np.float32, 1000, depth=4)
    ratio = f32["model_cells_per_s"] / f64["model_cells_per_s"]
    assert 1.9 < ratio < 2.2


def test_depth_hint_still_wins():
    info = _plan(wl.SUITE_2D[0], (8192, 8192), np.float64, 1000, depth=3)
    assert info["depth"] == 3


@pytest.mark.parametrize("idx", range(4), ids=[s.name for s in wl.SUITE_2D])
def test_shared_tiles_plan_like_a_full_device(idx):
    # A 1024^2 grid alone leaves most wave slots idle in its last round of
    # tiles, which favours shallow depths; planned for a batch (uniform tiles,
    # the slots shared with other jobs) the same grid takes the depth a grid
    # that fills the device would take.
    spec = wl.SUITE_2D[idx]
    alone = _plan(spec, (1024, 1024), np.float32, 400)
    shared = _plan(spec, (1024, 1024), np.float32, 400, seg_len=256, flags=st.STENCIL_FLAG_UNIFORM_TILES)
    full = _plan(spec, (8192, 8192), np.float32, 400)
    assert alone["depth"] < shared["depth"]
    assert abs(shared["depth"] - full["depth"]) <= 1


def test_shared_3d_tiles_plan_like_a_full_device():
    spec = wl.SUITE_3D[0]
    fl = st.STENCIL_FLAG_UNIFORM_TILES | st.STENCIL_FLAG_OVERLAPPED_TILING
    alone = _plan(spec, (64, 128, 128), np.float32, 400)
    shared = _plan(spec, (64, 128, 128), np.float32, 400, seg_len=64, flags=fl)
    full = _plan(spec, (512, 512, 512), np.float32, 400)
    assert alone["depth"] < shared["depth"] == full["depth"]


# depth caps of the fused batch kernel below the single-grid ones (its one
# register allocation for every variant): 2D radius-2 stars 7 / 6 (FP64 /
# FP32), 2D radius-3 stars 4, 2D radius-1 and -2 boxes 8 and 5
BATCH_CAPS = {(2, "star", 2): {np.float64: 7, np.float32: 6}, (2, "star", 3): {np.float64: 4, np.float32: 4},
              (2, "box", 1): {np.float64: 8, np.float32: 8}, (2, "box", 2): {np.float64: 5, np.float32: 5}}


def test_batch_describe_reports_the_batched_plan():
    # the 128-grid batch: every job planned as the batch runs it, never
    # shallower than the same grid planned alone (within the fused kernel's
    # caps), and never device-tiled
    probs = wl.batch_problems()
    deeper = 0
    for p in probs:
        for dt in (np.float64, np.float32):
            info = st.stencil_batch_describe(p.coeffs, p.spec.r, p.interior, dt, p.T)
            alone = _plan(p.spec, p.interior, dt, p.T, seed=0)
            cap = BATCH_CAPS.get((p.spec.ndim, p.spec.kind, p.spec.r), {}).get(dt, 99)
            assert info["scheme_name"] in ("blocked_2d", "blocked_3d")
            assert info["passes"] == -(-p.T // info["depth"])
            assert info["depth"] <= cap
            assert info["depth"] >= min(alone["depth"], cap) or p.T < alone["depth"]
            deeper += info["depth"] > alone["depth"]
    assert deeper > len(probs) // 2
    with pytest.raises(st.StencilError):
        st.stencil_batch_describe(probs[0].coeffs, probs[0].spec.r, probs[0].interior, np.float64, -1)


@pytest.mark.parametrize("ndim,kind,r", [(3, "box", 2), (3, "general", 2), (2, "general", 3), (2, "general", 4),
                                         (3, "star", 3)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_depth_hint_without_a_blocked_kernel(ndim, kind, r, dtype):
    # a variant with no blocked kernel for this dtype (compiled depth 0) takes
    # the plain kernel whatever depth is hinted, with every scheme flag; a
    # depth-0 candidate once reached the pass schedule and divided by zero
    shape = (13, 70, 140) if ndim == 3 else (150, 1100)
    w = wl.random_coeffs(ndim, "box" if kind == "general" else kind, r, 5).copy()
    if kind == "general":
        w[(0,) * ndim] = 0.0
    for depth in (0, 1, 3, 99):
        for flags in (0, st.STENCIL_FLAG_DEVICE_TILING, st.STENCIL_FLAG_OVERLAPPED_TILING):
            info = _plan_w(w, r, shape, dtype, 50, depth=depth, flags=flags)
            assert info["depth"] >= 1 and info["passes"] == -(-50 // info["depth"])
            if info["scheme_name"] == "naive":
                assert info["depth"] == 1


def _plan_w(w, r, shape, dtype, T, **kw):
    p = st.Plan(w, r, shape, dtype, T, flags=NC | kw.pop("flags", 0), **kw)
    info = p.info
    p.close()
    return info
