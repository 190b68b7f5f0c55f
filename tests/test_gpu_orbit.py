"""Moving detection point on the GPU, against the oracle.

Sec. IV.A divides the quasi-particle sample of a bin among the positions of a
spacecraft orbit (cosmica_job.orbit): particle i starts at position
i mod n_orbit, so each bin's flux is the average over the mission.  The
integrator's own device code runs in every test:

* a one-position orbit at the fixed injection point changes no bit;
* after one step every particle sits next to its own position;
* whole-path parity against the oracle for a polar (Ulysses-like) orbit,
  FP64 with the spherical 3D tolerances, mixed with the paired test;
* an orbit crossing into a heliosheath (positions beyond the shock);
* served results equal batch ones bit for bit.
"""
import math
import os

import numpy as np
import pytest

from paper_2502_06319_amd import cosmica as C
from tests.test_gpu_path import _compare_3d

pytestmark = pytest.mark.gpu

KEYS = ("hist", "flux", "flux_se", "mean_exit_time_s", "steps", "n_capped", "n_nan")


def _xyz(r, th, ph):
    return np.stack([r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)], -1)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_single_position_orbit_changes_nothing(eng, W, precision):
    job = W.c2_job(particles_per_bin=300, n_bins=4)
    h = job["helio"]
    one = W.with_orbit(job, [[h["r0_au"], h["theta0_rad"], h["phi0_rad"]]])
    a = eng.run(job, precision, exits=True)[0]
    b = eng.run(one, precision, exits=True)[0]
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    np.testing.assert_array_equal(a["exits"], b["exits"])


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_particles_start_at_their_own_position(eng, W, precision):
    orbit = np.array([[1.0, 0.6, 0.3], [20.0, 1.4, 2.0], [45.0, 2.5, 4.0], [70.0, 1.0, 5.5]])
    job = W.make_job(W.helio_3d([1.5e22] * 15, [400.0] * 15, [20.0] * 15, dt_max=5e3),
                     W.species("p"), [2.0, 9.0], 203)
    job["step_cap"] = 1
    g = eng.run(W.with_orbit(job, orbit), precision, exits=True)[0]
    ex = g["exits"]
    assert np.all(ex["n"] == 1) and np.all(ex["flags"] == 1)
    k = np.tile(np.arange(203) % 4, 2)
    x = _xyz(ex["r"], ex["theta"], ex["phi"])
    d = np.linalg.norm(x[:, None, :] - _xyz(*orbit.T)[None, :, :], axis=2)
    np.testing.assert_array_equal(np.argmin(d, axis=1), k)
    # one step spreads by ~1 AU at 2 GV and ~2.5 AU at 9 GV (dt = 5e3 s); the
    # positions are at least 19 AU apart
    assert np.all(d[np.arange(len(k)), k] < 12.0)


def test_polar_orbit_fp64_against_oracle(eng, orc, W, othreads):
    job = W.with_orbit(W.c2_job(particles_per_bin=480, n_bins=8), W.ulysses_like_orbit(24))
    overall, stats = _compare_3d(eng, orc, job, "fp64", othreads, "orbit-fp64")
    assert overall >= 0.90
    for same, dJ, se_pair, r, _ in stats:
        assert same >= 0.75
        assert abs(dJ) <= 0.5 * r["flux_se"]
        assert abs(dJ) <= 4.0 * se_pair + 1e-12 * r["flux"]


def test_polar_orbit_mixed_against_oracle(eng, orc, W, othreads):
    job = W.with_orbit(W.c2_job(particles_per_bin=960, n_bins=8), W.ulysses_like_orbit(24))
    overall, stats = _compare_3d(eng, orc, job, "mixed", othreads, "orbit-mixed")
    for same, dJ, se_pair, r, _ in stats:
        N = r["n_used"]
        assert abs(dJ) <= 4.0 * se_pair + 1e-12 * r["flux"]
        assert abs(dJ) <= max(r["flux_se"], r["flux"] / math.sqrt(N))


def test_orbit_into_the_heliosheath(eng, orc, W, othreads):
    """Positions on both sides of the termination shock (a Voyager-like
    probe), FP64 with the current sheet off: particle by particle."""
    job = W.c2_heliosheath_job(particles_per_bin=300, n_bins=6)
    job["helio"]["hcs"] = 0
    h = job["helio"]
    orbit = [[40.0, 1.3, 0.5], [70.0, 1.2, h["nose_phi_rad"]],
             [h["ts_tail_au"] + 5.0, math.pi - h["nose_theta_rad"], h["nose_phi_rad"] + math.pi]]
    p = orc.params(W.with_orbit(job, orbit))
    assert orc.locate(p, *orbit[2])[1] == C.REGION_HELIOSHEATH
    overall, stats = _compare_3d(eng, orc, W.with_orbit(job, orbit), "fp64", othreads,
                                 "orbit-hs-fp64")
    assert overall >= 0.95
    for same, dJ, se_pair, r, _ in stats:
        assert abs(dJ) <= 0.1 * r["flux_se"]


def test_served_orbit_equals_batch(W):
    old = os.environ.get("COSMICA_SLICE_STEPS")
    os.environ["COSMICA_SLICE_STEPS"] = "300"
    try:
        jobs = [W.with_orbit(W.c2_job(particles_per_bin=150, n_bins=3), W.earth_orbit(12)),
                W.with_orbit(W.c2_job(particles_per_bin=120, n_bins=2), W.ulysses_like_orbit(24))]
        jobs[1]["job_tag"] = 4
        with C.Engine(0) as e:
            tickets = [e.submit(j, "mixed", exits=True) for j in jobs]
            for t in tickets:
                assert t.wait(120000) == C.OK
            for j, t in zip(jobs, tickets):
                alone = e.run(j, "mixed", exits=True)[0]
                got = t.result()
                for k in KEYS:
                    np.testing.assert_array_equal(got[k], alone[k], err_msg=k)
    finally:
        if old is None:
            del os.environ["COSMICA_SLICE_STEPS"]
        else:
            os.environ["COSMICA_SLICE_STEPS"] = old
