"""Serving API argument checks (host only)."""
import numpy as np
import pytest

from paper_2305_07390_amd import stencil as st


@pytest.mark.parametrize("budget,slots,rounds", [(0, 4, 0), (1 << 30, 0, 0), (1 << 30, 4, 3)])
def test_create_rejects_bad_config(budget, slots, rounds):
    with pytest.raises(st.StencilError) as e:
        st.stencil_server_create(budget, slots, rounds_in_flight=rounds)
    assert e.value.status == st.STENCIL_ERR_INVALID


def test_null_arguments_rejected():
    lib = st.load_library()
    assert lib.stencil_server_create(None, None) == st.STENCIL_ERR_INVALID
    assert lib.stencil_server_submit(None, None, None, None) == st.STENCIL_ERR_INVALID
    assert lib.stencil_server_poll(None, 1, None, None, None) == st.STENCIL_ERR_INVALID
    assert lib.stencil_server_wait(None, 1, None, None) == st.STENCIL_ERR_INVALID
    assert lib.stencil_server_stats(None, None) == st.STENCIL_ERR_INVALID
    assert lib.stencil_server_destroy(None) == st.STENCIL_ERR_INVALID
