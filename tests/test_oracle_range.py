"""Pins of the oracle's exit histogram over the reached range.

The paper takes the largest exit energy of a sample to set the binning of
its exit histogram (Sec. IV.A).  The oracle's reading: equal bins in
ln(P_ex/P0) over [0, ln(P_max/P0)].  Pinned (P27) against numpy's own
histogram of the same logarithms, the maximum against numpy's, the count
total, and the degenerate cases; capped and non-finite records stay out.
"""
import math

import numpy as np
import pytest


def _records(orc, P, flags=None):
    rec = np.zeros(len(P), dtype=orc.EXIT_DTYPE)
    rec["P"] = P
    if flags is not None:
        rec["flags"] = flags
    return rec


@pytest.mark.parametrize("n_hist", [1, 7, 128, 1000])
def test_p27_equals_numpy_histogram_of_the_log_ratio(orc, n_hist):
    rng = np.random.default_rng(n_hist)
    P0 = 0.7
    P = P0 * np.exp(rng.gamma(2.0, 0.4, 5000))
    pm, hist = orc.exit_range(P0, _records(orc, P), n_hist)
    assert pm == P.max()
    ref, _ = np.histogram(np.log(P / P0), bins=n_hist, range=(0.0, math.log(P.max() / P0)))
    np.testing.assert_array_equal(hist, ref)
    assert hist.sum() == len(P) and hist[-1] >= 1  # the record at P_max is in the last bin


def test_p27_flagged_records_stay_out(orc):
    rng = np.random.default_rng(3)
    P0 = 2.0
    P = P0 * np.exp(rng.uniform(0.0, 1.0, 1000))
    flags = np.zeros(1000, dtype=np.uint32)
    flags[:10] = 1  # capped, with rigidities above every used one
    flags[10:20] = 2  # non-finite
    P[:10] = 1e3
    pm, hist = orc.exit_range(P0, _records(orc, P, flags), 16)
    used = P[20:]
    assert pm == used.max() and hist.sum() == 980
    ref, _ = np.histogram(np.log(used / P0), bins=16, range=(0.0, math.log(used.max() / P0)))
    np.testing.assert_array_equal(hist, ref)


def test_p27_degenerate_cases(orc):
    pm, hist = orc.exit_range(1.5, _records(orc, np.full(40, 1.5)), 8)  # no energy change
    assert pm == 1.5 and hist[0] == 40 and hist[1:].sum() == 0
    pm, hist = orc.exit_range(1.5, _records(orc, np.full(4, 2.0), np.ones(4, np.uint32)), 8)
    assert pm == 0.0 and hist.sum() == 0


def test_p27_on_propagated_exits(orc, W):
    job = W.c1_job(particles_per_bin=300)
    for r in orc.run_job(job, threads=8):
        rec = r["records"]
        pm, hist = orc.exit_range(r["P0"], rec, 64)
        assert pm == rec["P"].max() and pm >= r["P0"]
        assert hist.sum() == r["n_used"]
