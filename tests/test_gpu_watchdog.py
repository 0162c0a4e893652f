"""The watchdog of the persistent and batched launches, forced from the host:
with a zero time limit (STENCIL_WATCHDOG_US=0) the first wait that is not
already satisfied expires, every later item skips its work, the launch still
drains, and stencil_sync (or a persistent plan's execute) reports
STENCIL_ERR_TIMEOUT. The expiry stays with its own launch: the next run, with
the default limit, is clean and bit-identical to the oracle."""
import os

import numpy as np
import pytest

import oracle
from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture
def zero_watchdog():
    os.environ["STENCIL_WATCHDOG_US"] = "0"
    try:
        yield
    finally:
        os.environ.pop("STENCIL_WATCHDOG_US", None)


def test_persistent_expiry_is_reported_then_clean(zero_watchdog):
    import torch
    spec = wl.SUITE_2D[0]
    coeffs = wl.coeffs_for(spec, 5)
    u0 = wl.make_field((1024, 1024), 1, 5)
    x = torch.from_numpy(u0).cuda()
    y = torch.empty_like(x)
    # three passes of few tiles each: idle workgroups claim pass-1 items at
    # once and find pass 0 unfinished
    plan = st.Plan(coeffs, 1, (1024, 1024), np.float64, 36, flags=st.STENCIL_FLAG_PERSISTENT)
    assert plan.info["passes"] == 3
    print("persistent plan", plan.info, flush=True)
    with pytest.raises(st.StencilError) as e:
        plan.execute(x, y)
    assert e.value.status == st.STENCIL_ERR_TIMEOUT
    os.environ.pop("STENCIL_WATCHDOG_US")
    st.stencil_sync(st._stream_handle(None))  # nothing left to report
    plan.execute(x, y)
    np.testing.assert_array_equal(y.cpu().numpy(), oracle.sweep(coeffs, 1, u0, 36))
    plan.close()


def test_batch_expiry_is_reported_then_clean(zero_watchdog):
    import torch
    probs = wl.batch_problems(6, seed=12, side2d=(300, 700), side3d=(64, 90), t_range=(20, 40))
    xs = [torch.from_numpy(p.field()).cuda() for p in probs]
    ys = [torch.empty_like(x) for x in xs]
    print("batch", [(p.spec.name, p.interior, p.T) for p in probs], flush=True)
    st.run_batch(probs, xs, ys)
    with pytest.raises(st.StencilError) as e:
        st.stencil_sync(st._stream_handle(None))
    assert e.value.status == st.STENCIL_ERR_TIMEOUT
    os.environ.pop("STENCIL_WATCHDOG_US")
    st.run_batch(probs, xs, ys)
    st.stencil_sync(st._stream_handle(None))
    for p, x, y in zip(probs, xs, ys):
        np.testing.assert_array_equal(y.cpu().numpy(), oracle.sweep(p.coeffs, p.spec.r, p.field(), p.T))


@pytest.mark.parametrize("rounds", [1, 2], ids=["one_round", "two_rounds"])
def test_server_round_expiry_fails_its_request_then_clean(zero_watchdog, rounds):
    """A served request whose round's waits expire fails with
    STENCIL_ERR_TIMEOUT (the round's report word is read when the round is
    retired); the server clears the stream's report word, and the next
    request, run with the default limit, equals the oracle."""
    from paper_2305_07390_amd import serving
    spec = wl.SUITE_2D[0]
    coeffs = wl.coeffs_for(spec, 6)
    u0 = wl.make_field((1024, 1024), 1, 6)
    with serving.Server(hbm_budget_bytes=1 << 30, max_slots=4, quantum_passes=4,
                        rounds_in_flight=rounds) as srv:
        # three passes in one round: idle workgroups claim pass-1 items at
        # once and find pass 0 unfinished
        t = srv.submit(coeffs, 1, (1024, 1024), 36, u0)
        print("server request T=36 at 1024^2, zero watchdog", flush=True)
        with pytest.raises(st.StencilError) as e:
            srv.wait(t, np.empty_like(u0))
        assert e.value.status == st.STENCIL_ERR_TIMEOUT
        os.environ.pop("STENCIL_WATCHDOG_US")
        t = srv.submit(coeffs, 1, (1024, 1024), 36, u0)
        got = np.empty_like(u0)
        srv.wait(t, got)
        s = srv.stats()
    np.testing.assert_array_equal(got, oracle.sweep(coeffs, 1, u0, 36))
    assert s["failed"] == 1 and s["completed"] == 1
