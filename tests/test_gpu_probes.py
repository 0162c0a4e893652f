"""Microbenchmarks of the model's parameters on the GPU: plausible magnitudes,
and the neighbour-exchange probe reads back every payload word with its
round's value under both publication schemes (the scheme the 3D device-tiled
pass uses is mode 1)."""
import json

import pytest

from paper_2305_07390_amd import stencil as st

pytestmark = pytest.mark.gpu


def test_copy_bandwidth():
    b = st.stencil_probe_copy(1 << 30)
    print(json.dumps({"copy_GBs": b / 1e9}), flush=True)
    assert 1e12 < b < 1.2e13


def test_latencies():
    hbm = st.stencil_probe_latency(st.PROBE_HBM_LATENCY)
    lds = st.stencil_probe_latency(st.PROBE_LDS_LATENCY)
    fma = st.stencil_probe_latency(st.PROBE_FMA64_LATENCY)
    print(json.dumps({"hbm_ns": hbm * 1e9, "lds_ns": lds * 1e9, "fma64_ns": fma * 1e9}), flush=True)
    assert 1e-7 < hbm < 1e-5
    assert 1e-9 < lds < 1e-6
    assert 1e-10 < fma < 1e-7
    assert hbm > lds > fma


def test_lds_bandwidth():
    b = st.stencil_probe_lds_bandwidth()
    print(json.dumps({"lds_GBs": b / 1e9}), flush=True)
    assert 1e12 < b < 2e14


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("payload", [0, 8192])
def test_neighbor_sync_is_coherent(mode, payload):
    t, bad = st.stencil_probe_neighbor_sync(mode, rounds=2000, payload_bytes=payload)
    print(json.dumps({"mode": mode, "payload": payload, "us_per_round": t * 1e6, "mismatches": bad}),
          flush=True)
    assert bad == 0
    assert 0 < t < 1e-3


def test_calibrate_replaces_the_machine_parameters():
    try:
        m = st.stencil_machine_calibrate(st._stream_handle(None))
        print(json.dumps(m), flush=True)
        assert m == st.stencil_machine_get()
        assert 2e12 < m["hbm_bytes_per_s"] < 1.2e13
        assert 1e13 < m["lds_bytes_per_s"] < 2e14
        assert 1e-6 < m["grid_sync_s"] < 1e-4 and 1e-7 < m["neighbor_sync_s"] < 1e-4
        assert m["cus"] == 256
    finally:
        st.stencil_machine_set(None)
