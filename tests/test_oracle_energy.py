"""Pins of the oracle's energy form (Eq.(1), the form of Versions 0-3).

Rearranged into the backward form of Eq.(2), Eq.(1) advances the kinetic
energy T with dT = (1/3)(div V) alpha T ds and carries the loss
L = (div V)[1 - (1/3) d(alpha T)/dT] into the exponential weight of Eq.(4).
Along an exact path L ds is d ln(p E): with dp = (1/3)(div V) p ds,
d ln(pE) = (1 + beta^2) dp/p and 1 - (1/3)(1 + (M/E)^2) = (1 + beta^2)/3.
So exp(-sum L ds) -> p0 E0 / (p_ex E_ex), and the energy form's
J_mod(P0) = mean(beta0/beta_ex J_LIS(P_ex) exp(-loss)) reproduces the momentum
form's P0^2 mean(J_LIS(P_ex)/P_ex^2).  These tests check that identity, which
no formula of the oracle states:

  P21 no wind: no energy change and no loss, J = J_LIS(P0) exactly;
  P22 each particle's weight exp(-loss) equals p0 E0 / (p_ex E_ex) up to the
      Euler-Maruyama error, which falls in proportion to the step;
  P23 energy- and momentum-form spectra agree within the Monte Carlo error
      (the paper's version comparison, Sec. VIII, Fig. 5).
"""
import math

import numpy as np
import pytest

M_P = 0.93827208816


def _job(W, n=300, bins=6, scale=1.0, **kw):
    job = W.c2_job(particles_per_bin=n, n_bins=bins)
    h = job["helio"]
    h["dt_max_s"] *= scale
    h["dt_diff_frac"] *= scale
    h["dt_adv_frac"] *= scale
    h.update(kw)
    job["formulation"] = 1
    return job


def _dev(res, mass=M_P, Z=1):
    """exp(-loss) / (p0 E0 / (p_ex E_ex)) - 1 per particle, p = |Z| P."""
    out = []
    for r in res:
        rec, P0 = r["records"], r["P0"]
        ratio = (P0 * math.hypot(Z * P0, mass)) / (rec["P"] * np.hypot(Z * rec["P"], mass))
        out.append(np.exp(-rec["loss"]) / ratio - 1.0)
    return out


def test_p21_no_wind_no_energy_change(orc, W):
    h = W.helio_3d([1.5e22] * 3, [0.0] * 3, [30.0] * 3, drift=0, hcs=0, v_fast=0.0,
                   r_boundary=100.0)
    job = W.make_job(h, W.species("He4"), [0.3, 2.0, 40.0], 128)
    job["formulation"] = 1
    p = orc.params(job)
    for r in orc.run_job(job, threads=4):
        # the state is T; P = P(T(P0)) returns P0 up to the rounding of the two maps
        np.testing.assert_allclose(r["records"]["P"], r["P0"], rtol=1e-14)
        assert np.all(r["records"]["loss"] == 0.0)
        assert r["flux"] == pytest.approx(orc.lis(p, r["P0"]), rel=1e-12)


def test_p22_loss_weight_is_the_endpoint_ratio(orc, W):
    coarse = _dev(orc.run_job(_job(W), threads=8))
    fine = _dev(orc.run_job(_job(W, scale=0.25), threads=8))
    for c, f in zip(coarse, fine):
        assert np.abs(c).max() < 5e-2
        # first order in the step: a quarter of the step, about a quarter of the error
        assert 2.5 < np.median(np.abs(c)) / np.median(np.abs(f)) < 6.5
    # heavier nuclei, other rest energies: the same identity
    job = _job(W, n=200, bins=4)
    job["species"] = W.species("He3")
    for d in _dev(orc.run_job(job, threads=8), mass=W.species("He3")["mass_gev"], Z=2):
        assert np.abs(d).max() < 5e-2


def test_p23_energy_and_momentum_forms_agree(orc, W):
    job = _job(W, n=600, bins=6)
    e = orc.run_job(job, threads=8)
    m = orc.run_job(dict(job, formulation=0), threads=8)
    for a, b in zip(e, m):
        assert abs(a["flux"] - b["flux"]) <= 2.0 * b["flux_se"]
        if a["P0"] >= 1.0:
            assert abs(a["flux"] / b["flux"] - 1.0) < 1e-2


def test_energy_form_is_3d_only(orc, W):
    job = W.c1_job(particles_per_bin=4)
    job["formulation"] = 1
    with pytest.raises(ValueError):
        orc.run_job(job, threads=1)
