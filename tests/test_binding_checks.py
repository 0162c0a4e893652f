"""The Python binding refuses buffers that do not match a plan or request
before any pointer reaches the library (CPU only: the checks run first)."""
import numpy as np
import pytest
import torch

from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl


@pytest.fixture(scope="module")
def plan():
    p = st.Plan(wl.coeffs_for(wl.SUITE_2D[0], 1), 1, (300, 400), np.float64, 5)
    yield p
    p.close()


def test_padded_nbytes():
    assert st.padded_nbytes((300, 400), 1, np.float64) == 302 * 402 * 8
    assert st.padded_nbytes((3, 4, 5), 2, np.float32) == 7 * 8 * 9 * 4


def test_execute_rejects_wrong_dtype(plan):
    x = torch.zeros((302, 402), dtype=torch.float32)
    y = torch.zeros((302, 402), dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        plan.execute(x, y)


def test_execute_rejects_wrong_size(plan):
    x = torch.zeros((302, 401), dtype=torch.float64)
    with pytest.raises(ValueError, match="bytes"):
        plan.execute(x, torch.zeros((302, 402), dtype=torch.float64))
    with pytest.raises(ValueError, match="bytes"):
        plan.execute(torch.zeros(10, dtype=torch.float64), torch.zeros((302, 402), dtype=torch.float64))


def test_execute_rejects_non_contiguous(plan):
    x = torch.zeros((402, 302), dtype=torch.float64).t()
    with pytest.raises(ValueError, match="contiguous"):
        plan.execute(x, x)


def test_execute_rejects_host_tensor(plan):
    x = torch.zeros((302, 402), dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU"):
        plan.execute(x, x.clone())


def test_run_batch_rejects_mismatch():
    prob = wl.Problem(wl.SUITE_2D[0], wl.coeffs_for(wl.SUITE_2D[0], 1), (300, 400), 5, field_seed=1)
    good = torch.zeros((302, 402), dtype=torch.float64)
    with pytest.raises(ValueError, match="job 0 output"):
        st.run_batch([prob], [good], [torch.zeros((302, 402), dtype=torch.float32)])
    with pytest.raises(ValueError, match="job 0 input"):
        st.run_batch([prob], [torch.zeros(5, dtype=torch.float64)], [good])


def test_server_submit_rejects_wrong_host_size():
    coeffs = wl.coeffs_for(wl.SUITE_2D[0], 1)
    with pytest.raises(ValueError, match="bytes"):
        st.stencil_server_submit(0, coeffs, 1, (300, 400), 5, np.zeros((302, 401), dtype=np.float32))
    with pytest.raises(ValueError):
        st.stencil_server_submit(0, coeffs, 1, (300, 400), 5, np.zeros((302, 402), dtype=np.int32))


def test_server_poll_rejects_unknown_ticket_buffer():
    with pytest.raises(ValueError, match="unknown ticket"):
        st.stencil_server_poll(0, 12345, np.zeros(4, dtype=np.float32))
