"""Autotuner on the GPU: the chosen plan is one of the compiled variants, the
cache then drives plans without hints, and results do not depend on the choice."""
import numpy as np
import pytest

from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _clean_cache():
    st.stencil_tune_cache_clear()
    yield
    st.stencil_tune_cache_clear()


CASES = [
    ("2d5pt_star_r1", (1024, 1536), np.float64, 0),
    ("2d25pt_box_r2", (700, 1100), np.float32, 0),
    ("3d7pt_star_r1", (96, 128, 160), np.float64, 0),
    ("2d9pt_box_r1", (1024, 1024), np.float64, st.STENCIL_TUNE_BATCH),
    ("3d27pt_box_r1", (64, 96, 128), np.float32, st.STENCIL_TUNE_BATCH),
]


@pytest.mark.parametrize("name,interior,dtype,flags", CASES, ids=[c[0] + ("_batch" if c[3] else "") for c in CASES])
def test_tune_then_plan_uses_choice(name, interior, dtype, flags):
    import torch
    spec = {s.name: s for s in wl.ALL_STENCILS}[name]
    coeffs = wl.coeffs_for(spec, 77)
    res = st.stencil_tune(coeffs, spec.r, interior, dtype, flags)
    print(name, res, flush=True)
    assert res["from_cache"] == 0 and res["candidates"] >= 1
    assert res["depth"] >= 1 and res["seconds_per_step"] > 0
    again = st.stencil_tune(coeffs, spec.r, interior, dtype, flags)
    assert again["from_cache"] == 1 and again["depth"] == res["depth"]
    assert st.stencil_tune_lookup(coeffs, spec.r, interior, dtype, flags) == (res["depth"], res["seg_len"])

    T = 3 * res["depth"] + 1
    u0 = wl.make_field(interior, spec.r, seed=5, dtype=dtype)
    x = torch.from_numpy(u0).cuda()
    ref = torch.empty_like(x)
    p0 = st.Plan(coeffs, spec.r, interior, dtype, T, depth=1, flags=st.STENCIL_FLAG_NO_CACHE)
    p0.execute(x, ref)
    y = torch.empty_like(x)
    if flags & st.STENCIL_TUNE_BATCH:
        st.stencil_batch_submit([dict(coeffs=coeffs, radius=spec.r, interior=interior, dtype=dtype, T=T,
                                      in_ptr=x.data_ptr(), out_ptr=y.data_ptr())],
                                st._stream_handle())
        st.stencil_sync(st._stream_handle())
    else:
        p = st.Plan(coeffs, spec.r, interior, dtype, T)
        assert p.info["depth"] == min(res["depth"], T)
        if res["seg_len"]:
            assert p.info["seg_len"] == res["seg_len"]
        p.execute(x, y)
        p.close()
    torch.cuda.synchronize()
    p0.close()
    assert torch.equal(y, ref)


def test_tune_rejects_shape_without_blocked_kernel():
    spec = wl.SUITE_2D[0]
    with pytest.raises(st.StencilError) as e:
        st.stencil_tune(wl.coeffs_for(spec, 1), spec.r, (40, 40), np.float64)
    assert e.value.status == st.STENCIL_ERR_UNSUPPORTED
