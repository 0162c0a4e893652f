"""Parity at the sizes the benchmark times, in the launch configuration it
times: the 8192^2 FP64 2D suite and the 512^3 FP64 3D suite with the planner's
default plans (as the benchmark builds them), run for T = 2t + rem steps so
that full-depth passes, a remainder pass and an odd pass count all occur, and
the 128-grid FP64 batch at its drawn step counts. Every output cell is
compared with the oracle, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _bench_plan_T(prob, dtype=np.float64):
    """Depth of the benchmark's plan for this problem, and a T of 2 full passes
    plus a shorter one."""
    full = st.Plan(prob.coeffs, prob.spec.r, prob.interior, dtype, prob.T)
    d = full.info["depth"]
    info = full.info
    full.close()
    rem = max(1, d // 2) if d > 1 else 0
    return d, 2 * d + rem, info


def _run(prob, T, dtype=np.float64):
    import torch
    u0 = prob.field(dtype)
    x = torch.from_numpy(u0).cuda()
    y = torch.full_like(x, float("nan"))
    plan = st.Plan(prob.coeffs, prob.spec.r, prob.interior, dtype, T)
    info = plan.info
    plan.execute(x, y)
    st.stencil_sync(st._stream_handle(None))
    got = y.cpu().numpy()
    plan.close()
    del x, y
    torch.cuda.empty_cache()
    return u0, got, info


@pytest.mark.parametrize("idx", range(4), ids=[s.name for s in wl.SUITE_2D])
def test_suite_2d_8192_fp64(idx):
    prob = wl.suite_2d_problems(8192, 1000)[idx]
    d, T, binfo = _bench_plan_T(prob)
    print(f"{prob.spec.name}: bench plan depth {d} tiles {binfo['tiles']} seg {binfo['seg_len']}; T = {T}",
          flush=True)
    u0, got, info = _run(prob, T)
    assert info["depth"] == d and info["tiles"] == binfo["tiles"] and info["seg_len"] == binfo["seg_len"]
    assert info["passes"] == 3
    ref = oracle.sweep(prob.coeffs, prob.spec.r, u0, T)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("idx", range(3), ids=[s.name for s in wl.SUITE_3D])
def test_suite_3d_512_fp64(idx):
    prob = wl.suite_3d_problems(512, 200)[idx]
    d, T, binfo = _bench_plan_T(prob)
    print(f"{prob.spec.name}: bench plan {binfo['scheme_name']} depth {d} tiles {binfo['tiles']}; T = {T}",
          flush=True)
    u0, got, info = _run(prob, T)
    assert info["depth"] == d and info["scheme"] == binfo["scheme"]
    ref = oracle.sweep(prob.coeffs, prob.spec.r, u0, T)
    np.testing.assert_array_equal(got, ref)


def test_batch_128_grids_fp64():
    import torch
    probs = wl.batch_problems()
    xs = [torch.from_numpy(p.field()).cuda() for p in probs]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    print(f"batch: {len(probs)} grids, {sum(p.updates for p in probs):.3e} updates", flush=True)
    st.run_batch(probs, xs, ys)
    st.stencil_sync(st._stream_handle(None))
    del xs
    for k, (p, y) in enumerate(zip(probs, ys)):
        got = y.cpu().numpy()
        ref = oracle.sweep(p.coeffs, p.spec.r, p.field(), p.T)
        assert np.array_equal(got, ref), (k, p.spec.name, p.interior, p.T)
