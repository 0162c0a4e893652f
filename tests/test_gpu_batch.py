"""Batched persistent execution: every job of a mixed batch equals its own
single-grid run and the oracle, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl
from tests.gpu_util import gpu_sweep

pytestmark = pytest.mark.gpu


def _mixed_problems(dtype, seed=5):
    rng = np.random.default_rng(seed)
    probs = []
    kinds = [(2, "star", 1), (2, "box", 1), (2, "star", 3), (2, "box", 2), (3, "star", 1),
             (3, "box", 1), (3, "star", 2)]
    for g in range(14):
        ndim, kind, r = kinds[g % len(kinds)]
        spec = wl.StencilSpec(f"{ndim}d_{kind}_r{r}", ndim, kind, r)
        if ndim == 2:
            interior = (int(rng.integers(200, 700)), int(rng.integers(256, 900)))
            T = int(rng.integers(3, 40))
        else:
            interior = (int(rng.integers(10, 40)), int(rng.integers(64, 100)), int(rng.integers(64, 110)))
            T = int(rng.integers(2, 9))
        coeffs = wl.coeffs_for(spec, 100 + g)
        probs.append(wl.Problem(spec, coeffs, interior, T, field_seed=200 + g, tag=g))
    return probs


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_batch_equals_single_and_oracle(dtype):
    import torch
    probs = _mixed_problems(dtype)
    fields = [p.field(dtype) for p in probs]
    xs = [torch.from_numpy(f).cuda() for f in fields]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    status = st.run_batch(probs, xs, ys)
    assert all(s == st.STENCIL_OK for s in status), status
    st.stencil_sync(torch.cuda.current_stream().cuda_stream)
    for p, f, x, y in zip(probs, fields, xs, ys):
        got = y.cpu().numpy()
        assert np.array_equal(x.cpu().numpy(), f), "input modified"
        single = gpu_sweep(p.coeffs, p.spec.r, f, p.T)
        assert np.array_equal(got, single), (p.spec.name, p.interior, p.T, "batch != single run")
        ref = oracle.sweep(p.coeffs, p.spec.r, f, p.T)
        assert np.array_equal(got, ref), (p.spec.name, p.interior, p.T, "batch != oracle")


def test_batch_repeat_is_deterministic():
    import torch
    probs = _mixed_problems(np.float64, seed=9)[:7]
    xs = [torch.from_numpy(p.field()).cuda() for p in probs]
    outs = []
    for _ in range(2):
        ys = [torch.empty_like(x) for x in xs]
        st.run_batch(probs, xs, ys)
        st.stencil_sync(torch.cuda.current_stream().cuda_stream)
        outs.append([y.cpu().numpy() for y in ys])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_batch_reports_invalid_jobs():
    import torch
    probs = _mixed_problems(np.float64, seed=11)[:3]
    xs = [torch.from_numpy(p.field()).cuda() for p in probs]
    ys = [torch.empty_like(x) for x in xs]
    specs = []
    for p, x, y in zip(probs, xs, ys):
        specs.append(dict(coeffs=p.coeffs, radius=p.spec.r, interior=p.interior, dtype=x.dtype,
                          T=p.T, in_ptr=x.data_ptr(), out_ptr=y.data_ptr()))
    specs[1]["T"] = -3  # invalid: reported, skipped
    status = st.stencil_batch_submit(specs, torch.cuda.current_stream().cuda_stream)
    st.stencil_sync(torch.cuda.current_stream().cuda_stream)
    assert status[1] == st.STENCIL_ERR_INVALID and status[0] == 0 and status[2] == 0
    for k in (0, 2):
        ref = oracle.sweep(probs[k].coeffs, probs[k].spec.r, probs[k].field(), probs[k].T)
        assert np.array_equal(ys[k].cpu().numpy(), ref)


def test_batch_fp64_3d_radius2_jobs_fused_apart():
    """FP64 3D radius-2 stars take the auxiliary batch kernel (several jobs of
    different shapes and T next to a 2D job); each equals the oracle."""
    import torch
    spec = wl.StencilSpec("3d_star_r2", 3, "star", 2)
    shapes = [((20, 64, 70), 4), ((33, 70, 96), 6), ((12, 80, 64), 3), ((40, 64, 130), 5)]
    probs = [wl.Problem(spec, wl.coeffs_for(spec, 300 + g), shp, T, field_seed=310 + g, tag=g)
             for g, (shp, T) in enumerate(shapes)]
    s2 = wl.StencilSpec("2d_star_r1", 2, "star", 1)
    probs.append(wl.Problem(s2, wl.coeffs_for(s2, 320), (300, 600), 13, field_seed=321, tag=9))
    fields = [p.field(np.float64) for p in probs]
    xs = [torch.from_numpy(f).cuda() for f in fields]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    status = st.run_batch(probs, xs, ys)
    assert all(s == st.STENCIL_OK for s in status), status
    st.stencil_sync(torch.cuda.current_stream().cuda_stream)
    for p, f, y in zip(probs, fields, ys):
        ref = oracle.sweep(p.coeffs, p.spec.r, f, p.T)
        assert np.array_equal(y.cpu().numpy(), ref), (p.spec.name, p.interior, p.T)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_batch_mixes_alone_jobs(dtype):
    """Jobs without a batched variant (T = 0 copy, a grid narrower than one wave
    tile, a 3D radius-2 box) run after the persistent launches, next to fused
    jobs; each equals the oracle."""
    import torch
    specs = [
        (wl.StencilSpec("2d_star_r1", 2, "star", 1), (40, 300), 0),      # copy
        (wl.StencilSpec("2d_star_r1", 2, "star", 1), (50, 60), 7),       # plain kernel
        (wl.StencilSpec("3d_box_r2", 3, "box", 2), (10, 20, 24), 3),     # no blocked 3D variant
        (wl.StencilSpec("2d_box_r1", 2, "box", 1), (260, 700), 11),      # fused
        (wl.StencilSpec("3d_star_r1", 3, "star", 1), (18, 70, 80), 6),   # fused
    ]
    probs = [wl.Problem(s, wl.coeffs_for(s, 400 + g), shp, T, field_seed=410 + g, tag=g)
             for g, (s, shp, T) in enumerate(specs)]
    fields = [p.field(dtype) for p in probs]
    xs = [torch.from_numpy(f).cuda() for f in fields]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    status = st.run_batch(probs, xs, ys)
    assert all(s == st.STENCIL_OK for s in status), status
    st.stencil_sync(torch.cuda.current_stream().cuda_stream)
    for p, f, y in zip(probs, fields, ys):
        ref = oracle.sweep(p.coeffs, p.spec.r, f, p.T)
        assert np.array_equal(y.cpu().numpy(), ref), (p.spec.name, p.interior, p.T)


def test_batch_three_groups_side_by_side():
    """One submission with FP32 jobs, fused FP64 jobs and FP64 3D radius-2
    stars: three persistent launches (FP32 fused, FP64 fused, FP64 auxiliary)
    one after another on the caller's stream. Every job equals the oracle,
    twice in a row."""
    import torch
    cases = [
        (wl.StencilSpec("2d_star_r1", 2, "star", 1), (300, 520), 17, np.float32),
        (wl.StencilSpec("3d_star_r1", 3, "star", 1), (24, 70, 90), 5, np.float32),
        (wl.StencilSpec("2d_box_r2", 2, "box", 2), (260, 640), 9, np.float64),
        (wl.StencilSpec("3d_box_r1", 3, "box", 1), (20, 66, 80), 4, np.float64),
        (wl.StencilSpec("3d_star_r2", 3, "star", 2), (30, 64, 100), 6, np.float64),
        (wl.StencilSpec("3d_star_r2", 3, "star", 2), (14, 72, 64), 3, np.float64),
    ]
    probs = [wl.Problem(s, wl.coeffs_for(s, 500 + g), shp, T, field_seed=510 + g, tag=g)
             for g, (s, shp, T, _) in enumerate(cases)]
    fields = [p.field(dt) for p, (_, _, _, dt) in zip(probs, cases)]
    refs = [oracle.sweep(p.coeffs, p.spec.r, f, p.T) for p, f in zip(probs, fields)]
    xs = [torch.from_numpy(f).cuda() for f in fields]
    for _ in range(2):
        ys = [torch.full_like(x, float("nan")) for x in xs]
        status = st.run_batch(probs, xs, ys)
        assert all(s == st.STENCIL_OK for s in status), status
        st.stencil_sync(torch.cuda.current_stream().cuda_stream)
        for p, y, ref in zip(probs, ys, refs):
            assert np.array_equal(y.cpu().numpy(), ref), (p.spec.name, p.interior, p.T)
