"""Pins of the oracle's re-weighting of stored exit records.

The paths do not depend on the local interstellar spectrum: it only enters
the weight of Eq.(4).  So exit records can be re-weighted with any number of
other spectra (the fitting use of Sec. VIII), each tabulated as ln J on a
uniform ln P grid and interpolated linearly in log-log.

  P24 a power law is a straight line in log-log, so any tabulation of the
      job's own spectrum reproduces the bin's flux and standard error to
      rounding (momentum and energy form, extrapolation included);
  P25 a broken power law with its break on a knot is also exact: the
      re-weighted flux equals the mean of its analytic weights;
  P26 re-weighting to another spectral index equals propagating again with
      that index.
"""
import math

import numpy as np
import pytest

LNP0, DLNP, NK = math.log(0.05), 0.25, 40  # knots from 0.05 GV to ~900 GV


def _table(norm, index, lnP0=LNP0, dlnP=DLNP, nk=NK):
    lnP = lnP0 + dlnP * np.arange(nk)
    return math.log(norm) - index * lnP


@pytest.mark.parametrize("formulation", [0, 1])
def test_p24_own_power_law_reproduces_the_reduction(orc, W, formulation):
    job = W.c2_job(particles_per_bin=300, n_bins=4)
    job["formulation"] = formulation
    p = orc.params(job)
    sp = job["species"]
    for r in orc.run_job(job, threads=8):
        # a narrow table: most exits need the extended end segments
        for lnP0, nk in ((LNP0, NK), (math.log(1.0), 4)):
            f, se = orc.reweight_bin(p, r["P0"], r["records"], lnP0, DLNP,
                                     _table(sp["lis_norm"], sp["lis_index"], lnP0, DLNP, nk))
            assert f[0] == pytest.approx(r["flux"], rel=1e-12)
            assert se[0] == pytest.approx(r["flux_se"], rel=1e-9)


def test_p25_broken_power_law_on_a_knot(orc, W):
    job = W.c2_job(particles_per_bin=400, n_bins=3)
    p = orc.params(job)
    kb = 12  # break at knot 12
    Pb = math.exp(LNP0 + DLNP * kb)
    lnP = LNP0 + DLNP * np.arange(NK)
    lnJ = np.where(lnP < LNP0 + DLNP * kb, math.log(2e4) - 2.6 * lnP,
                   math.log(2e4) - 2.6 * math.log(Pb) - 3.1 * (lnP - math.log(Pb)))
    for r in orc.run_job(job, threads=8):
        rec = r["records"]
        P = rec["P"]
        J = np.where(P < Pb, 2e4 * P ** -2.6, 2e4 * Pb ** -2.6 * (P / Pb) ** -3.1)
        w = r["P0"] ** 2 * J / P ** 2
        f, se = orc.reweight_bin(p, r["P0"], rec, LNP0, DLNP, lnJ)
        assert f[0] == pytest.approx(w.mean(), rel=1e-12)
        assert se[0] == pytest.approx(w.std(ddof=1) / math.sqrt(len(w)), rel=1e-9)


@pytest.mark.parametrize("formulation", [0, 1])
def test_p26_reweighting_equals_propagating_with_that_spectrum(orc, W, formulation):
    job = W.c2_job(particles_per_bin=300, n_bins=4)
    job["formulation"] = formulation
    p = orc.params(job)
    indices = (2.4, 2.78, 3.2)
    tables = np.stack([_table(1.9e4, g) for g in indices])
    base = orc.run_job(job, threads=8)
    for g_i, g in enumerate(indices):
        other = dict(job, species=dict(job["species"], lis_index=g))
        for r0, r1 in zip(base, orc.run_job(other, threads=8)):
            np.testing.assert_array_equal(r0["records"]["P"], r1["records"]["P"])
            f, se = orc.reweight_bin(p, r0["P0"], r0["records"], LNP0, DLNP, tables)
            assert f[g_i] == pytest.approx(r1["flux"], rel=1e-12)
            assert se[g_i] == pytest.approx(r1["flux_se"], rel=1e-9)
