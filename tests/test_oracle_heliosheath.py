"""Pins of the oracle's nose-squashed heliosphere and heliosheath.

The paper splits the heliosphere into an inner heliosphere and a heliosheath,
both squashed toward the nose (Sec. II.B), without giving a shape.  The
reading implemented: the heliopause and the termination shock are spheres
whose centres sit behind the Sun, against the nose direction, fixed by their
distances toward the nose (Rn) and the tail (Rt); the heliosheath between them
is one more parameter region.  Each pin compares the oracle with something the
geometry or the mathematics fixes, never with its own formulas:

  P13 boundary distance along a direction at angle psi from the nose, from the
      law of cosines: R(psi) = -d cos(psi) + sqrt(a^2 - d^2 sin^2(psi)),
      a = (Rn + Rt)/2, d = (Rt - Rn)/2; the region flips to the heliosheath at
      the termination shock's R(psi).
  P14 pure isotropic diffusion inside an off-centre sphere:
      E[tau] = (a^2 - |x0 - c|^2) / (6 kappa), with the discrete-monitoring
      shift of a; injections toward the nose and toward the tail tell the
      centre's side apart.
  P15 pure diffusion with a heliosheath of a different kappa (concentric
      spheres): E[tau] from kappa (u'' + 2u'/r) = -1 in each zone with u and
      u' continuous at the shock (the radial scale density r^-2 does not
      depend on kappa), u = 0 at the heliopause.
  P16 a heliosheath whose parameters equal the single shell's changes no bit.
"""
import math

import numpy as np
import pytest
from scipy import constants as sc

AU_CM = sc.au * 100.0
M_P = 0.93827208816


def _beta(P, mass=M_P):
    return P / math.sqrt(P * P + mass * mass)


def _unit(theta, phi):
    return np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi),
                     math.cos(theta)])


def _R_of(psi, Rn, Rt):
    a, d = 0.5 * (Rn + Rt), 0.5 * (Rt - Rn)
    return -d * math.cos(psi) + math.sqrt(a * a - d * d * math.sin(psi) ** 2)


def _iso_helio(W, kappa0=1.5e22, n_regions=1, r_boundary=100.0, dt_max=1e3):
    h = W.helio_3d([kappa0] * n_regions, [0.0] * n_regions, [10.0] * n_regions, drift=0,
                   hcs=0, kperp_over_kpar=1.0, v_fast=0.0, r_boundary=r_boundary,
                   dt_max=dt_max, dt_adv_frac=0.0)
    return h


# --------------------------------------------------------------------------
# P13
# --------------------------------------------------------------------------
def test_p13_boundary_and_shock_surfaces(orc, W):
    nose_t, nose_p = math.radians(95.0), math.radians(40.0)
    h = W.with_heliosheath(W.helio_3d([1e22] * 15, [400.0] * 15, [20.0] * 15), ts_nose=84.0,
                           ts_tail=110.0, hp_nose=120.0, hp_tail=170.0, kappa0_hs=0.5e22,
                           v_hs=150.0, tilt_hs_deg=20.0, nose_theta=nose_t, nose_phi=nose_p)
    p = orc.params(W.make_job(h, W.species("p"), [1.0], 1))
    n_hat = _unit(nose_t, nose_p)
    rng = np.random.default_rng(3)
    dirs = [(nose_t, nose_p), (math.pi - nose_t, nose_p + math.pi)]
    for _ in range(200):
        dirs.append((math.acos(rng.uniform(-1, 1)), rng.uniform(0, 2 * math.pi)))
    for th, ph in dirs:
        psi = math.acos(max(-1.0, min(1.0, float(_unit(th, ph) @ n_hat))))
        R_hp, R_ts = _R_of(psi, 120.0, 170.0), _R_of(psi, 84.0, 110.0)
        out_in, k_in = orc.locate(p, R_hp * (1 - 1e-7), th, ph)
        out_out, k_out = orc.locate(p, R_hp * (1 + 1e-7), th, ph)
        assert not out_in and out_out
        assert k_in == 15 and k_out == 15  # beyond the shock: the heliosheath
        _, k_before = orc.locate(p, R_ts * (1 - 1e-7), th, ph)
        _, k_after = orc.locate(p, R_ts * (1 + 1e-7), th, ph)
        assert 0 <= k_before <= 14 and k_after == 15
    # the extremes are the nose and tail distances themselves
    assert _R_of(0.0, 120.0, 170.0) == pytest.approx(120.0)
    assert _R_of(math.pi, 120.0, 170.0) == pytest.approx(170.0)
    # shells: equal widths up to the shock's nose distance
    for r, k in ((0.5 * 84.0 / 15, 0), (84.0 / 15 * 7.5, 7), (83.9, 14)):
        assert orc.locate(p, r, nose_t, nose_p)[1] == k


def test_p13_spherical_boundary_is_the_plain_radius_test(orc, W):
    h = _iso_helio(W, r_boundary=100.0)
    p = orc.params(W.make_job(h, W.species("p"), [1.0], 1))
    for th, ph in ((0.3, 1.0), (2.0, 5.0), (math.pi / 2, 0.0)):
        assert orc.locate(p, 100.0, th, ph) == (True, 0)
        assert orc.locate(p, np.nextafter(100.0, 0.0), th, ph) == (False, 0)


# --------------------------------------------------------------------------
# P14
# --------------------------------------------------------------------------
@pytest.mark.parametrize("toward", ["nose", "tail"])
def test_p14_exit_time_from_off_centre_sphere(orc, W, toward):
    nose_t, nose_p = math.radians(95.0), math.radians(40.0)
    Rn, Rt, r0 = 60.0, 100.0, 30.0
    a, d = 0.5 * (Rn + Rt), 0.5 * (Rt - Rn)
    h = _iso_helio(W, r_boundary=Rt)
    h["r_boundary_nose_au"] = Rn
    h["nose_theta_rad"], h["nose_phi_rad"] = nose_t, nose_p
    if toward == "nose":
        h["r0_au"], h["theta0_rad"], h["phi0_rad"] = r0, nose_t, nose_p
    else:
        h["r0_au"], h["theta0_rad"], h["phi0_rad"] = r0, math.pi - nose_t, nose_p + math.pi
    P0, N, dt = 2.0, 2048, 1e3
    res = orc.run_job(W.make_job(h, W.species("p"), [P0], N), threads=8)[0]
    kap = 1.5e22 / AU_CM**2 * _beta(P0) * P0
    x0 = r0 * _unit(h["theta0_rad"], h["phi0_rad"])
    c = -d * _unit(nose_t, nose_p)
    dist2 = float((x0 - c) @ (x0 - c))
    assert math.sqrt(dist2) == pytest.approx(r0 + d if toward == "nose" else abs(r0 - d))
    shift = 0.5826 * math.sqrt(2.0 * kap * dt)
    pred = ((a + shift) ** 2 - dist2) / (6.0 * kap)
    t = res["records"]["t"]
    se = t.std(ddof=1) / math.sqrt(N)
    assert abs(t.mean() - pred) <= 3.0 * se
    # every exit lies on or outside the boundary, within one step of it
    rec = res["records"]
    for e in rec[:200]:
        x = e["r"] * _unit(e["theta"], e["phi"])
        dc = math.sqrt(float((x - c) @ (x - c)))
        assert a <= dc < a + 6.0 * math.sqrt(2.0 * kap * dt)


# --------------------------------------------------------------------------
# P15
# --------------------------------------------------------------------------
def _two_zone_tau(k1, k2, R1, R2, r0):
    B2 = R1**3 / 3.0 * (1.0 / k1 - 1.0 / k2)
    A2 = R2**2 / (6.0 * k2) - B2 / R2
    A1 = A2 - R1**2 / (6.0 * k2) + B2 / R1 + R1**2 / (6.0 * k1)
    return A1 - r0**2 / (6.0 * k1)


def test_p15_exit_time_with_a_slower_heliosheath(orc, W):
    R1, R2, P0, N, dt = 50.0, 100.0, 2.0, 2048, 2e3
    h = W.with_heliosheath(_iso_helio(W, r_boundary=R2, dt_max=dt), ts_nose=R1, ts_tail=R1,
                           hp_nose=R2, hp_tail=R2, kappa0_hs=0.5e22, v_hs=0.0, tilt_hs_deg=10.0)
    res = orc.run_job(W.make_job(h, W.species("p"), [P0], N), threads=8)[0]
    b = _beta(P0) * P0 / AU_CM**2
    k1, k2 = 1.5e22 * b, 0.5e22 * b
    shift = 0.5826 * math.sqrt(2.0 * k2 * dt)
    pred = _two_zone_tau(k1, k2, R1, R2 + shift, 1.0)
    t = res["records"]["t"]
    se = t.std(ddof=1) / math.sqrt(N)
    assert abs(t.mean() - pred) <= 3.0 * se
    # the slower heliosheath is visible: one kappa throughout would be ~half as long
    assert t.mean() > 1.5 * (R2**2 - 1.0) / (6.0 * k1)
    assert _two_zone_tau(k1, k1, R1, R2, 1.0) == pytest.approx((R2**2 - 1.0) / (6.0 * k1))


# --------------------------------------------------------------------------
# P16
# --------------------------------------------------------------------------
def test_p16_heliosheath_with_the_shell_parameters_changes_nothing(orc, W):
    base = W.helio_3d([1.2e22], [450.0], [25.0], v_fast=450.0, r_boundary=100.0)
    hs = W.with_heliosheath(base, ts_nose=60.0, ts_tail=80.0, hp_nose=100.0, hp_tail=100.0,
                            kappa0_hs=1.2e22, v_hs=450.0, tilt_hs_deg=25.0,
                            nose_theta=math.radians(95.0), nose_phi=1.0)
    for P0 in (0.5, 5.0):
        a = orc.run_job(W.make_job(base, W.species("p"), [P0], 200), threads=8)[0]["records"]
        b = orc.run_job(W.make_job(hs, W.species("p"), [P0], 200), threads=8)[0]["records"]
        for f in ("P", "t", "n", "r", "theta", "phi"):
            np.testing.assert_array_equal(a[f], b[f])
    # and a different heliosheath does change the paths
    hs2 = dict(hs, kappa0_hs_cm2_s=0.6e22)
    c = orc.run_job(W.make_job(hs2, W.species("p"), [5.0], 200), threads=8)[0]["records"]
    assert not np.array_equal(a["t"], c["t"])
