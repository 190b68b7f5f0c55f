"""Pins of the oracle's moving detection point.

Sec. IV.A divides the quasi-particle sample of a bin among the positions of a
spacecraft orbit, so the fluxes integrate over the mission.  The reading
implemented: K positions at equal time steps, particle i starting at position
i mod K; the bin's flux is the mean over all its particles.

  P17 a one-position orbit at the fixed injection point changes no bit;
  P18 after one step every particle sits next to its own orbit position;
  P19 pure isotropic diffusion from positions at radii r_k:
      E[tau] = mean_k (R^2 - r_k^2) / (6 kappa), with the discrete-monitoring
      shift of R (positions at one radius alone would give one term);
  P20 Kepler positions at equal times sweep equal areas (second law), and
      the radii span perihelion to aphelion.
"""
import math

import numpy as np
import pytest
from scipy import constants as sc

AU_CM = sc.au * 100.0
M_P = 0.93827208816


def _beta(P, mass=M_P):
    return P / math.sqrt(P * P + mass * mass)


def _xyz(r, th, ph):
    return np.stack([r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)], -1)


def test_p17_single_position_orbit_changes_nothing(orc, W):
    job = W.c2_job(particles_per_bin=200, n_bins=3)
    h = job["helio"]
    one = W.with_orbit(job, [[h["r0_au"], h["theta0_rad"], h["phi0_rad"]]])
    a = orc.run_job(job, threads=8)
    b = orc.run_job(one, threads=8)
    for x, y in zip(a, b):
        for f in ("P", "t", "n", "r", "theta", "phi"):
            np.testing.assert_array_equal(x["records"][f], y["records"][f])


@pytest.mark.parametrize("model", [0, 1])
def test_p18_particles_start_at_their_own_position(orc, W, model):
    orbit = np.array([[1.0, 0.6, 0.3], [20.0, 1.4, 2.0], [45.0, 2.5, 4.0], [70.0, 1.0, 5.5]])
    # one step spreads by sqrt(2 kappa dt) ~ 1 AU at dt = 5e3 s, far below the
    # spacing of the positions
    if model == 0:
        job = W.make_job(W.helio_1d(dt_max=5e3), W.species("p"), [2.0], 101)
    else:
        job = W.make_job(W.helio_3d([1.5e22] * 15, [400.0] * 15, [20.0] * 15, dt_max=5e3),
                         W.species("p"), [2.0], 101)
    job["step_cap"] = 1
    rec = orc.run_job(W.with_orbit(job, orbit), threads=4)[0]["records"]
    assert np.all(rec["n"] == 1) and np.all(rec["flags"] == 1)
    k = np.arange(101) % 4
    if model == 0:
        d = np.abs(rec["r"][:, None] - orbit[None, :, 0])
    else:
        x = _xyz(rec["r"], rec["theta"], rec["phi"])
        d = np.linalg.norm(x[:, None, :] - _xyz(*orbit.T)[None, :, :], axis=2)
    np.testing.assert_array_equal(np.argmin(d, axis=1), k)
    assert np.all(d[np.arange(101), k] < 5.0)


def test_p19_exit_time_averages_over_the_orbit(orc, W):
    radii = np.array([1.0, 20.0, 40.0, 60.0, 80.0])
    orbit = np.stack([radii, np.full(5, 1.2), np.linspace(0.0, 5.0, 5)], 1)
    R, P0, dt = 100.0, 2.0, 1e3
    h = W.helio_3d([1.5e22], [0.0], [10.0], drift=0, hcs=0, kperp_over_kpar=1.0, v_fast=0.0,
                   r_boundary=R, dt_max=dt, dt_adv_frac=0.0)
    N = 5 * 800
    res = orc.run_job(W.with_orbit(W.make_job(h, W.species("p"), [P0], N), orbit),
                      threads=8)[0]
    kap = 1.5e22 / AU_CM**2 * _beta(P0) * P0
    Rs = R + 0.5826 * math.sqrt(2.0 * kap * dt)
    t = res["records"]["t"]
    k = np.arange(N) % 5
    for j in range(5):  # each position on its own
        tj = t[k == j]
        assert abs(tj.mean() - (Rs**2 - radii[j] ** 2) / (6 * kap)) <= 3.5 * tj.std(ddof=1) / math.sqrt(len(tj))
    pred = np.mean((Rs**2 - radii**2) / (6 * kap))
    assert abs(t.mean() - pred) <= 3.0 * t.std(ddof=1) / math.sqrt(N)


def test_p20_kepler_positions_at_equal_times(W):
    n, a, e = 360, 3.37, 0.603
    o = W.kepler_orbit(n, a, e, 79.1, arg_peri_deg=-90.0)
    x = _xyz(*o.T)
    # equal areas in equal times: |x_k x x_{k+1}| is (nearly) constant
    areas = np.linalg.norm(np.cross(x, np.roll(x, -1, axis=0)), axis=1)
    assert areas.std() / areas.mean() < 2e-3
    # samples sit half a step off perihelion and aphelion
    assert o[:, 0].min() == pytest.approx(a * (1 - e), rel=1e-3)
    assert o[:, 0].max() == pytest.approx(a * (1 + e), rel=1e-3)
    # the orbit plane is inclined 79.1 deg to the solar equator
    nrm = np.cross(x[0], x[n // 4])
    assert math.degrees(math.acos(abs(nrm[2]) / np.linalg.norm(nrm))) == pytest.approx(79.1, abs=1e-6)
