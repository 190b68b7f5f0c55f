"""Host logic of the parameter-scan driver (no device work): grid expansion,
parameter application, the power-law tables and the chi^2 fit."""
import math

import numpy as np
import pytest

from paper_2502_06319_amd import scan as S


def test_power_law_tables_are_exact_lines():
    lnJ, lnP0, dlnP = S.power_law_tables([1.9e4, 2e4], [2.7, 3.0], n_knots=10)
    assert lnJ.shape == (4, 10)
    lnP = lnP0 + dlnP * np.arange(10)
    np.testing.assert_allclose(lnJ[3], math.log(2e4) - 3.0 * lnP, rtol=0, atol=1e-12)


def test_apply_scales_every_kappa(W):
    h = W.with_heliosheath(W.c2_job(particles_per_bin=1, n_bins=1)["helio"], 85, 100, 120, 160,
                           0.5e22, 150.0, 20.0)
    g = S._apply(h, {"kappa0_scale": 2.0, "tilt_deg": 33.0, "polarity": -1})
    np.testing.assert_allclose(g["kappa0_cm2_s"], 2.0 * np.array(h["kappa0_cm2_s"]))
    assert g["kappa0_hs_cm2_s"] == 2.0 * h["kappa0_hs_cm2_s"]
    assert g["tilt_deg"] == [33.0] * 15 and g["polarity"] == -1
    assert h["polarity"] == 1  # the base is untouched


def test_fit_finds_the_generating_point_and_averages():
    rng = np.random.default_rng(1)
    pts = [{"a": a} for a in (0.5, 1.0, 1.5, 2.0)]
    P = np.array([1.0, 2.0, 4.0, 8.0])
    model = lambda a, g: 100.0 * P ** -g * np.exp(-a / P)
    gs = (2.5, 2.7, 2.9)
    flux = np.array([[model(p["a"], g) for g in gs] for p in pts])
    res = S.ScanResult(pts, np.zeros((3, 2)), flux, 1e-3 * flux, P)
    obs = model(1.5, 2.7)
    out = S.fit(res, obs * (1 + 1e-3 * rng.standard_normal(4)), 1e-2 * obs,
                lis_params=np.array(gs)[:, None])
    assert out["best_point"] == {"a": 1.5} and out["best_lis"] == 1
    assert out["mean"]["a"] == pytest.approx(1.5, abs=0.05)
    assert out["mean"]["lis"][0] == pytest.approx(2.7, abs=0.02)
