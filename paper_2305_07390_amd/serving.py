"""Serving front end: a thin Python handle over the library's native server
(``stencil_server_*``) and an open-loop driver that submits requests at given
arrival times (Poisson arrivals) while collecting results.

All scheduling, admission, device memory and batching happen in the native
server; this module only marshals arguments and drives arrivals."""
from __future__ import annotations

import threading
import time

import numpy as np

from . import stencil as st


class Server:
    """Context-managed native server on one device."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int, quantum_passes: int = 0, device: int = 0,
                 round_target_s: float = 0.0, rounds_in_flight: int = 0):
        self.handle = st.stencil_server_create(hbm_budget_bytes, max_slots, quantum_passes, device,
                                               round_target_s, rounds_in_flight)

    def submit(self, coeffs, radius: int, interior, T: int, field: np.ndarray) -> int:
        return st.stencil_server_submit(self.handle, coeffs, radius, interior, T, field)

    def submit_problem(self, problem, field: np.ndarray, T: int | None = None) -> int:
        return self.submit(problem.coeffs, problem.spec.r, problem.interior,
                           problem.T if T is None else T, field)

    def poll(self, ticket: int, out: np.ndarray | None = None):
        return st.stencil_server_poll(self.handle, ticket, out)

    def wait(self, ticket: int, out: np.ndarray | None = None) -> float:
        return st.stencil_server_wait(self.handle, ticket, out)

    def stats(self) -> dict:
        return st.stencil_server_stats(self.handle)

    def close(self):
        if self.handle:
            st.stencil_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def serve_open_loop(server: Server, requests, arrivals, keep_results: bool = False,
                    on_result=None) -> dict:
    """Submit ``requests`` (tuples ``(problem, field, T)``) at ``arrivals``
    (seconds from the start, non-decreasing) from a submitter thread, and
    collect every result in submission order on the calling thread.

    Returns ``{"latency_s": [...], "arrival_latency_s": [...], "results":
    [...] or None, "rejected": [...], "submit_lag_s": max lateness of a
    submission, "stats": server stats}``. ``latency_s`` is the server's own
    figure (from the submit call to the end of the round that completes the
    request); ``arrival_latency_s`` adds the request's lag from its scheduled
    arrival to that call, so a driver that falls behind does not hide queueing.
    ``on_result(index, array)`` is called for each collected result."""
    n = len(requests)
    tickets = [None] * n
    errors = [None] * n
    ready = [threading.Event() for _ in range(n)]
    lags = [0.0] * n
    t0 = time.perf_counter()

    def submitter():
        for k, ((prob, field, T), at) in enumerate(zip(requests, arrivals)):
            delay = at - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            lags[k] = max(0.0, time.perf_counter() - t0 - at)
            try:
                tickets[k] = server.submit_problem(prob, field, T)
            except st.StencilError as e:
                errors[k] = e
            ready[k].set()

    th = threading.Thread(target=submitter, daemon=True)
    th.start()
    latencies, arrival_lat, results, rejected = [], [], [] if keep_results else None, []
    for k in range(n):
        ready[k].wait()
        if tickets[k] is None:
            rejected.append((k, errors[k]))
            continue
        field = requests[k][1]
        out = np.empty_like(field)
        latencies.append(server.wait(tickets[k], out))
        arrival_lat.append(latencies[-1] + lags[k])
        if keep_results:
            results.append(out)
        if on_result is not None:
            on_result(k, out)
    th.join()
    return {"latency_s": latencies, "arrival_latency_s": arrival_lat, "results": results,
            "rejected": rejected, "submit_lag_s": max(lags) if lags else 0.0,
            "stats": server.stats()}
