"""The serving statistics of bench.py (latency percentiles, the warm-up window,
shedding at the cut and the steady rate), driven on the CPU by a stand-in
engine whose requests finish a fixed time after they are submitted."""
import os
import sys
import threading
import time

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2502_06319_amd import cosmica as C  # noqa: E402

STEPS_PER_REQUEST = 1000


class _Ticket:
    def __init__(self, eng, admitted):
        self.eng = eng
        self.t_done = time.perf_counter() + eng.latency if admitted else None
        self.cancelled = False

    def state(self):
        if self.cancelled or (self.t_done is not None and time.perf_counter() >= self.t_done):
            return 2
        return 1 if self.t_done is not None else 0

    def poll(self):
        if self.cancelled:
            return True, C.ECANCELED
        if self.t_done is not None and time.perf_counter() >= self.t_done:
            return True, C.OK
        return False, C.OK

    def cancel(self):
        if self.state() != 2:
            self.cancelled = True
        return C.OK

    def result(self):
        return {"steps": np.array([STEPS_PER_REQUEST // 2, STEPS_PER_REQUEST // 2], np.uint64)}


class _Engine:
    """Admits the first `admit` requests (each done `latency` seconds after its
    submission); later ones wait for admission until cancelled."""

    def __init__(self, latency, admit=None):
        self.latency = latency
        self.admit = admit
        self.n = 0
        self.lock = threading.Lock()

    def submit(self, job, precision):
        with self.lock:
            self.n += 1
            admitted = self.admit is None or self.n <= self.admit
        return _Ticket(self, admitted)


def test_warmup_window_and_percentiles():
    eng = _Engine(latency=0.02)
    out = bench.serve(eng, 1.0, 40.0, "mixed", seed=7, warmup_s=0.4)
    reqs = bench.W.c5_requests(seed=7, rate_hz=40.0, duration_s=1.0)
    measured = sum(1 for r in reqs if r["arrival_s"] >= 0.4)
    assert out["requests"] == len(reqs)
    assert out["completed"] == len(reqs)  # early requests are served, not counted
    assert out["measured_requests"] == measured > 0
    # latency = the stand-in's 20 ms, plus submission and poll granularity
    # (generous: the host may be busy)
    assert 0.018 <= out["p50_latency_s"] <= 0.25
    assert out["p50_latency_s"] <= out["p90_latency_s"] <= out["p99_latency_s"] <= out["max_latency_s"]
    # throughput over the measured window only
    # ("seconds" is rounded to 10 ms)
    assert out["steps_per_s"] == pytest.approx(measured * STEPS_PER_REQUEST / out["seconds"],
                                               rel=0.02)
    assert out["spectra_per_hour"] == pytest.approx(measured / out["seconds"] * 3600.0, rel=0.02)


def test_cut_sheds_waiting_requests_and_reports_the_steady_rate():
    eng = _Engine(latency=0.05, admit=12)
    out = bench.serve(eng, 1.0, 40.0, "mixed", seed=9, cut_at=1.0, poll_s=0.005)
    reqs = bench.W.c5_requests(seed=9, rate_hz=40.0, duration_s=1.0)
    assert out["completed"] == 12
    assert out["cancelled_unadmitted"] == len(reqs) - 12
    assert out["steady_window_s"] == [0.25, 1.0]
    # the 12 admitted requests finish 50 ms after their arrivals: those that
    # finish inside [0.25, 1.0) s make up the steady rate
    arrivals = [r["arrival_s"] for r in reqs[:12]]
    # (completions are seen up to a poll late; 0.1 s of slack for a busy host)
    in_window = sum(1 for a in arrivals if 0.25 <= a + 0.05 < 1.0 - 0.1)
    near_edge = sum(1 for a in arrivals if 0.25 - 0.1 <= a + 0.05 < 0.25 or 1.0 - 0.1 <= a + 0.05 < 1.0)
    assert in_window <= out["steady_requests"] <= in_window + near_edge
    assert out["steady_steps_per_s"] == pytest.approx(
        out["steady_requests"] * STEPS_PER_REQUEST / 0.75)
