"""stencil_run_noalloc against stencil_run, through the C ABI: two calls in a
row on one GPU, the second on a smaller grid (the scratch region keeps the
first call's contents), each bit-identical to stencil_run on the same input,
for 2D and 3D, FP64 and FP32, and a single-pass plan larger than the region
(it needs no workspace). A plan whose workspace exceeds the region is
rejected before any device work."""
import numpy as np
import pytest

from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _pair(spec, interior, T, dtype, seed):
    import torch
    coeffs = wl.coeffs_for(spec, seed)
    u0 = wl.make_field(interior, spec.r, seed).astype(dtype)
    x = torch.from_numpy(u0).cuda()
    ya = torch.full_like(x, float("nan"))
    yb = torch.full_like(x, float("nan"))
    sh = st._stream_handle(None)
    print(f"{spec.name} {interior} T={T} {np.dtype(dtype).name}", flush=True)
    st.stencil_run(coeffs, spec.r, interior, dtype, T, x.data_ptr(), ya.data_ptr(), sh)
    st.stencil_run_noalloc(coeffs, spec.r, interior, dtype, T, x.data_ptr(), yb.data_ptr(), sh)
    st.stencil_sync(sh)
    return ya.cpu().numpy(), yb.cpu().numpy()


CASES = [
    # (spec, larger interior, smaller interior, T)
    (wl.SUITE_2D[0], (1000, 900), (300, 260), 37),
    (wl.SUITE_2D[3], (700, 640), (200, 300), 11),
    (wl.SUITE_3D[0], (64, 70, 96), (40, 36, 64), 9),
    (wl.SUITE_3D[1], (50, 40, 70), (20, 20, 64), 5),
]


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0].name for c in CASES])
def test_noalloc_equals_run_twice(case, dtype):
    spec, big, small, T = case
    for k, interior in enumerate((big, small)):
        ref, got = _pair(spec, interior, T, dtype, 40 + k)
        assert np.array_equal(got, ref), (spec.name, interior, T)


def test_single_pass_plan_beyond_region():
    # 3000 x 3000 FP64 is 72 MB padded, beyond the region, but T below the
    # depth is one pass and needs no workspace
    ref, got = _pair(wl.SUITE_2D[0], (3000, 3000), 5, np.float64, 7)
    assert np.array_equal(got, ref)


def test_workspace_beyond_region_is_rejected():
    import torch
    spec = wl.SUITE_2D[0]
    interior = (3000, 3000)
    x = torch.zeros((3002, 3002), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(st.StencilError) as e:
        st.stencil_run_noalloc(wl.coeffs_for(spec, 1), spec.r, interior, np.float64, 100, x.data_ptr(),
                               y.data_ptr(), st._stream_handle(None))
    assert e.value.status == st.STENCIL_ERR_INVALID
    assert "scratch" in str(e.value)
