"""Serving loop on the GPU: every served result equals the same request run
alone (bit for bit: quanta of passes are the same arithmetic), admission keeps
device memory within the budget and resident requests within the slots, and
the reported percentiles match the latencies returned."""
import math

import numpy as np
import pytest

from paper_2305_07390_amd import serving
from paper_2305_07390_amd import stencil as st
from paper_2305_07390_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _alone(prob, field, T):
    import torch
    x = torch.from_numpy(field).cuda()
    y = torch.empty_like(x)
    p = st.Plan(prob.coeffs, prob.spec.r, prob.interior, field.dtype, T)
    p.execute(x, y)
    torch.cuda.synchronize()
    p.close()
    return y.cpu().numpy()


def _small_requests(n, seed, dtype):
    reqs, arr = wl.serving_requests(n, rate_hz=400.0, seed=seed, pool=8, dtype=dtype,
                                    side2d=(256, 700), side3d=(64, 80), t_range=(1, 40))
    return reqs, arr


@pytest.mark.parametrize("rounds", [1, 2], ids=["one_round", "two_rounds"])
@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["f32", "f64"])
def test_served_results_equal_alone(dtype, rounds):
    reqs, arr = _small_requests(24, seed=21, dtype=dtype)
    # one pass per request per round, so requests take several rounds and
    # overlap with later arrivals (with two rounds in flight, also with the
    # round enqueued behind theirs)
    with serving.Server(hbm_budget_bytes=8 << 30, max_slots=16, quantum_passes=1,
                        rounds_in_flight=rounds) as srv:
        out = serving.serve_open_loop(srv, reqs, arr, keep_results=True)
    assert not out["rejected"]
    s = out["stats"]
    print(dtype.__name__, {k: s[k] for k in ("completed", "rounds", "max_active", "p50_s", "p99_s")}, flush=True)
    assert s["completed"] == len(reqs) and s["failed"] == 0
    assert s["rounds"] >= 2 and s["max_active"] >= 2  # requests did share rounds
    for (prob, field, T), got in zip(reqs, out["results"]):
        np.testing.assert_array_equal(got, _alone(prob, field, T))


@pytest.mark.parametrize("rounds", [1, 2], ids=["one_round", "two_rounds"])
def test_burst_with_T0_and_naive_shapes(rounds):
    spec = wl.SUITE_2D[1]
    coeffs = wl.coeffs_for(spec, 3)
    shapes = [(40, 50), (300, 520), (257, 1031)]  # the first has no blocked variant
    with serving.Server(hbm_budget_bytes=1 << 30, max_slots=8, quantum_passes=1,
                        rounds_in_flight=rounds) as srv:
        tickets, fields = [], []
        for k, (shape, T) in enumerate(zip(shapes + shapes, [0, 7, 33, 5, 0, 19])):
            f = wl.make_field(shape, spec.r, seed=40 + k, dtype=np.float64)
            fields.append((shape, f, T))
            tickets.append(srv.submit(coeffs, spec.r, shape, T, f))
        for (shape, f, T), t in zip(fields, tickets):
            got = np.empty_like(f)
            lat = srv.wait(t, got)
            assert lat > 0
            prob = wl.Problem(spec, coeffs, shape, T, field_seed=0)
            np.testing.assert_array_equal(got, _alone(prob, f, T) if T else f)
        with pytest.raises(st.StencilError):
            srv.wait(tickets[0])  # collected tickets are forgotten


@pytest.mark.parametrize("rounds", [1, 2], ids=["one_round", "two_rounds"])
def test_admission_respects_budget_and_slots(rounds):
    spec = wl.SUITE_2D[0]
    coeffs = wl.coeffs_for(spec, 9)
    shape = (1024, 1024)
    grid_bytes = (1024 + 2) ** 2 * 8
    # two resident grids plus one batch workspace per round in flight
    need = (2 + rounds) * ((grid_bytes + 255) // 256 * 256)
    budget = 2 * need + need // 2  # room for two resident requests
    with serving.Server(hbm_budget_bytes=budget, max_slots=8, quantum_passes=1,
                        rounds_in_flight=rounds) as srv:
        with pytest.raises(st.StencilError) as e:
            srv.submit(coeffs, spec.r, (2048, 2048), 10, wl.make_field((2048, 2048), 1, 1))
        assert e.value.status == st.STENCIL_ERR_BUDGET
        f = wl.make_field(shape, spec.r, seed=2)
        tickets = [srv.submit(coeffs, spec.r, shape, 60, f) for _ in range(6)]
        ref = _alone(wl.Problem(spec, coeffs, shape, 60, field_seed=2), f, 60)
        for t in tickets:
            got = np.empty_like(f)
            srv.wait(t, got)
            np.testing.assert_array_equal(got, ref)
        s = srv.stats()
    assert s["rejected"] == 1 and s["completed"] == 6
    assert s["hbm_peak"] <= budget and s["max_active"] <= 2


def test_work_share_quantum_equals_alone():
    """Rounds of a fair share of 5 ms of work per request: same results."""
    reqs, arr = _small_requests(16, seed=44, dtype=np.float32)
    with serving.Server(hbm_budget_bytes=8 << 30, max_slots=16, round_target_s=0.005) as srv:
        out = serving.serve_open_loop(srv, reqs, arr, keep_results=True)
    assert out["stats"]["completed"] == len(reqs)
    for (prob, field, T), got in zip(reqs, out["results"]):
        np.testing.assert_array_equal(got, _alone(prob, field, T))


def test_percentiles_match_latencies():
    reqs, arr = _small_requests(30, seed=33, dtype=np.float32)
    with serving.Server(hbm_budget_bytes=4 << 30, max_slots=32) as srv:
        out = serving.serve_open_loop(srv, reqs, arr)
    lat = sorted(out["latency_s"])
    s = out["stats"]
    rank = lambda p: lat[max(0, math.ceil(p * len(lat)) - 1)]
    assert s["p50_s"] == pytest.approx(rank(0.5), abs=1e-3)
    assert s["p99_s"] == pytest.approx(rank(0.99), abs=1e-3)
    assert s["cell_updates"] == sum(p.cells * T for p, _, T in reqs)


@pytest.mark.parametrize("rounds", [1, 2], ids=["one_round", "two_rounds"])
def test_large_T0_request_returns_its_input(rounds):
    """A T = 0 request runs as a device copy in a round, ordered after its
    upload: a grid large enough that the upload takes a while comes back
    unchanged."""
    spec = wl.SUITE_2D[0]
    coeffs = wl.coeffs_for(spec, 3)
    f = wl.make_field((4096, 4096), 1, seed=71, dtype=np.float32)
    g = wl.make_field((300, 400), 1, seed=72, dtype=np.float32)
    with serving.Server(hbm_budget_bytes=4 << 30, max_slots=4, quantum_passes=1, rounds_in_flight=rounds) as srv:
        t0 = srv.submit(coeffs, 1, (4096, 4096), 0, f)
        t1 = srv.submit(coeffs, 1, (300, 400), 5, g)
        out0 = np.empty_like(f)
        srv.wait(t0, out0)
        out1 = np.empty_like(g)
        srv.wait(t1, out1)
    np.testing.assert_array_equal(out0, f)
    np.testing.assert_array_equal(out1, _alone(spec_problem(spec, coeffs, (300, 400)), g, 5))


def spec_problem(spec, coeffs, interior):
    return wl.Problem(spec, coeffs, interior, 0, field_seed=0)
