"""The nose-squashed heliosphere with a heliosheath on the GPU, against the oracle.

Sec. II.B divides the heliosphere into an inner heliosphere and a heliosheath,
both squashed toward the nose.  The library's reading (cosmica.h): the
heliopause and the termination shock are off-centre spheres set by their nose
and tail distances, and beyond the shock the heliosheath's own parameters
apply.  These tests run the integrator's own device code:

* region and exit decisions at points (cosmica_probe_locate) equal the
  oracle's away from the surfaces (within rounding of them either side is
  right);
* local coefficients inside the heliosheath equal the oracle's to the
  tolerances of the other coefficient tests;
* whole-path parity: FP64 particle by particle with the current sheet off,
  and statistically (paired and two-sample) with it on, where the wound
  heliosheath sheet amplifies rounding; mixed with the tolerances of the
  spherical 3D test;
* a spherical job in a launch that runs the surface-testing kernel is bitwise
  what the plain kernel gives;
* served results equal the batch ones bit for bit.
"""
import math

import numpy as np
import pytest

from paper_2502_06319_amd import cosmica as C
from tests.test_gpu_path import _compare_3d
from tests.test_gpu_rows import TOLS, _oracle_fields, _ratios

pytestmark = pytest.mark.gpu

KEYS = ("hist", "flux", "flux_se", "mean_exit_time_s", "steps", "n_capped", "n_nan")


def _unit(theta, phi):
    return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)],
                    -1)


def _R_of(cpsi, Rn, Rt):
    a, d = 0.5 * (Rn + Rt), 0.5 * (Rt - Rn)
    return -d * cpsi + np.sqrt(a * a - d * d * (1.0 - cpsi * cpsi))


@pytest.mark.parametrize("precision,gap", [("fp64", 1e-7), ("mixed", 1e-4)])
def test_locate_matches_oracle(eng, orc, W, precision, gap):
    job = W.c2_heliosheath_job(particles_per_bin=1, n_bins=1)
    h = job["helio"]
    p = orc.params(job)
    rng = np.random.default_rng(5)
    n = 600
    th = np.arccos(rng.uniform(-1.0, 1.0, n))
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    cpsi = _unit(th, ph) @ _unit(h["nose_theta_rad"], h["nose_phi_rad"])
    R_hp = _R_of(cpsi, h["r_boundary_nose_au"], h["r_boundary_au"])
    R_ts = _R_of(cpsi, h["ts_nose_au"], h["ts_tail_au"])
    # points just either side of both surfaces, and anywhere in between
    r = np.concatenate([R_hp * (1 - gap), R_hp * (1 + gap), R_ts * (1 - gap), R_ts * (1 + gap),
                        rng.uniform(0.5, 1.1, n) * R_hp])
    th, ph = np.tile(th, 5), np.tile(ph, 5)
    far = (np.abs(r / np.tile(R_hp, 5) - 1) > 0.5 * gap) & (np.abs(r / np.tile(R_ts, 5) - 1) >
                                                            0.5 * gap)
    r, th, ph = r[far], th[far], ph[far]
    region, outside = eng.probe_locate(job, np.stack([r, th, ph], 1), precision)
    want = [orc.locate(p, *q) for q in zip(r, th, ph)]
    np.testing.assert_array_equal(outside, [w[0] for w in want])
    np.testing.assert_array_equal(region, [w[1] for w in want])
    assert 0.2 < outside.mean() < 0.6
    assert np.sum(region == C.REGION_HELIOSHEATH) > 500


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_heliosheath_coefficients_match_oracle(eng, orc, W, precision):
    job = W.c2_heliosheath_job(particles_per_bin=1, n_bins=1)
    h = job["helio"]
    p = orc.params(job)
    rng = np.random.default_rng(12)
    n = 400
    pts = np.stack([np.exp(rng.uniform(math.log(0.1), math.log(100.0), n)),
                    rng.uniform(h["ts_tail_au"] + 0.5, h["r_boundary_au"], n),
                    rng.uniform(0.05, math.pi - 0.05, n), rng.uniform(0.0, 2 * math.pi, n)], 1)
    g = eng.probe_coeffs(job, pts, precision)
    o, extra = _oracle_fields(orc, p, pts)
    assert all(orc.coeffs_3d(p, *q)["region"] == C.REGION_HELIOSHEATH for q in pts[:20])
    # the heliosheath's kappa0 sets k_par there
    np.testing.assert_allclose(g[:, 15], o[:, 15], rtol=1e-6 if precision == "mixed" else 1e-12)
    worst, p99 = TOLS[precision]
    for name, rat in _ratios(g, o, extra, pts, h["kperp_over_kpar"]).items():
        i = int(np.argmax(rat))
        print(f"heliosheath {precision} {name}: max {rat[i]:.2e} p99 {np.percentile(rat, 99):.2e}",
              flush=True)
        assert rat[i] <= worst, name
        assert np.percentile(rat, 99) <= p99, name


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_slow_wind_coefficients_match_oracle(eng, orc, W, precision):
    """Winds of 20 km/s in the outer five shells and in the heliosheath: the
    current sheet's phase Omega r / V_s reaches ~3,700 rad (~590 revolutions)
    at the heliopause's tail.  The binary32 kernel reduces it to one revolution
    in FP64 before its sine, so the coefficients match the oracle at any wind
    speed, inside the sheet layer too."""
    job = W.c2_heliosheath_job(particles_per_bin=1, n_bins=1)
    h = job["helio"]
    h["v_hs_km_s"] = 20.0
    h["v_slow_km_s"] = list(h["v_slow_km_s"][:10]) + [20.0] * 5
    p = orc.params(job)
    rng = np.random.default_rng(13)
    n = 300
    pts = np.stack([np.exp(rng.uniform(math.log(0.1), math.log(100.0), n)),
                    rng.uniform(80.0, h["r_boundary_au"] - 0.5, n),
                    rng.uniform(0.05, math.pi - 0.05, n), rng.uniform(0.0, 2 * math.pi, n)], 1)
    # points inside the sheet layer: the sheet's colatitude by bisection on the
    # sign of the polarity factor, then a few sheet widths either side
    sheet = []
    for _ in range(80):
        P = math.exp(rng.uniform(math.log(0.2), math.log(50.0)))
        r = rng.uniform(80.0, h["r_boundary_au"] - 0.5)
        ph = rng.uniform(0.0, 2 * math.pi)
        lo, hi = 0.05, math.pi - 0.05
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if orc.coeffs_3d(p, P, r, mid, ph)["Hw"] > 0 else (lo, mid)
        c = orc.coeffs_3d(p, P, r, lo, ph)
        rl = 0.0222974 * P / c["Bmag_nT"]
        sheet.append([P, r, min(max(lo + rng.uniform(-2.0, 2.0) * 2.0 * rl / r, 0.05),
                                math.pi - 0.05), ph])
    pts = np.concatenate([pts, np.array(sheet)])
    assert orc.coeffs_3d(p, 1.0, 180.0, 1.5, 0.0)["V"] * 1.495978707e8 == pytest.approx(20.0)
    g = eng.probe_coeffs(job, pts, precision)
    o, extra = _oracle_fields(orc, p, pts)
    worst, p99 = TOLS[precision]
    if precision == "fp64":
        # the sheet's phase (~3,000 rad here) carries an FP64 rounding of
        # ~1e-16 of itself, against a sheet only ~1e-4 rad wide at low rigidity
        worst, p99 = 1e-8, 2e-9
    else:
        # Inside the sheet layer: at 20 km/s and low rigidity the sheet is only
        # ~2e-4 rad wide, while a binary32 longitude in [4, 2 pi) resolves
        # 4.8e-7 rad, so the polarity factor carries ~1e-3 of rounding there
        worst, p99 = 2e-2, 5e-3
    for name, rat in _ratios(g, o, extra, pts, h["kperp_over_kpar"]).items():
        i = int(np.argmax(rat))
        print(f"slow wind {precision} {name}: max {rat[i]:.2e} at P,r,th,ph={pts[i]} "
              f"p99 {np.percentile(rat, 99):.2e}", flush=True)
        assert rat[i] <= worst, name
        assert np.percentile(rat, 99) <= p99, name
    assert np.sum(np.abs(o[-80:, 9]) < 0.9) >= 20  # the sheet points are in the layer


def test_heliosheath_fp64_path_by_path_without_the_sheet(eng, orc, W, othreads):
    """Geometry, shock, heliosheath parameters and gradient-curvature drift,
    particle by particle: with the current sheet off, FP64 paths coincide."""
    job = W.c2_heliosheath_job(particles_per_bin=400, n_bins=8)
    job["helio"]["hcs"] = 0
    overall, stats = _compare_3d(eng, orc, job, "fp64", othreads, "hs-nosheet-fp64")
    assert overall >= 0.95
    for same, dJ, se_pair, r, _ in stats:
        assert same >= 0.90
        assert abs(dJ) <= 0.1 * r["flux_se"]


def test_heliosheath_fp64_against_oracle(eng, orc, W, othreads):
    """With the current sheet, the heliosheath's slow wind winds the sheet to
    about 3 rad per AU and paths that meet it amplify rounding: one ulp of the
    injection radius changes the step count of 15-35 % of the oracle's own
    particles.  Parity is then the paired and two-sample statistics."""
    job = W.c2_heliosheath_job(particles_per_bin=400, n_bins=8)
    overall, stats = _compare_3d(eng, orc, job, "fp64", othreads, "hs-fp64")
    for same, dJ, se_pair, r, _ in stats:
        assert abs(dJ) <= 4.0 * se_pair + 1e-12 * r["flux"]
        assert abs(dJ) <= 4.0 * math.sqrt(2.0) * r["flux_se"]


def test_heliosheath_mixed_against_oracle(eng, orc, W, othreads):
    job = W.c2_heliosheath_job(particles_per_bin=1000, n_bins=8)
    overall, stats = _compare_3d(eng, orc, job, "mixed", othreads, "hs-mixed")
    for same, dJ, se_pair, r, _ in stats:
        N = r["n_used"]
        assert abs(dJ) <= 4.0 * se_pair + 1e-12 * r["flux"]
        assert abs(dJ) <= max(r["flux_se"], r["flux"] / math.sqrt(N))


def test_heliosheath_changes_the_spectrum(eng, W):
    """The heliosheath slows the particles down: longer exit times, lower flux
    at low rigidity, than the same shells out to a spherical boundary."""
    hs = W.c2_heliosheath_job(particles_per_bin=800, n_bins=4)
    sph = W.c2_job(particles_per_bin=800, n_bins=4)
    a = eng.run(hs, "mixed")[0]
    b = eng.run(sph, "mixed")[0]
    assert np.all(a["mean_exit_time_s"] > b["mean_exit_time_s"])
    assert a["flux"][0] < b["flux"][0]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_spherical_job_is_unchanged_in_a_shaped_launch(eng, W, precision):
    sph = W.c2_job(particles_per_bin=300, n_bins=5)
    hs = W.c2_heliosheath_job(particles_per_bin=100, n_bins=3)
    hs["job_tag"] = 5
    alone = eng.run(sph, precision, exits=True)[0]
    mixed = eng.run([hs, sph], precision, exits=True)[1]
    for k in KEYS:
        np.testing.assert_array_equal(mixed[k], alone[k], err_msg=k)
    np.testing.assert_array_equal(mixed["exits"], alone["exits"])


def test_served_heliosheath_equals_batch(W):
    import os

    old = os.environ.get("COSMICA_SLICE_STEPS")
    os.environ["COSMICA_SLICE_STEPS"] = "300"
    try:
        jobs = [W.c2_heliosheath_job(particles_per_bin=150, n_bins=3),
                W.c2_job(particles_per_bin=150, n_bins=3)]
        jobs[1]["job_tag"] = 9
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
