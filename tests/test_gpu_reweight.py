"""Re-weighting of stored exit records on the GPU (cosmica_plan_reweight), and
the parameter-scan driver built on it.

The spectrum enters only the weight of Eq.(4), so exits can be re-weighted
with other local interstellar spectra (Sec. VIII's fitting use).  Tests:

* radial model, FP64: paths equal the oracle's particle by particle, so the
  re-weighted fluxes of 24 spectra (power laws, broken, curved) equal the
  oracle's own re-weighting to 1e-12;
* 3D energy form, FP64, current sheet off: paths coincide, fluxes to 1e-6;
* the job's own power law reproduces the plan's flux (both precisions and
  formulations); many spectra at once equal one at a time;
* a scan over kappa0 scale and LIS index recovers the parameters of a
  synthetic observation.
"""
import math

import numpy as np
import pytest

from paper_2502_06319_amd import cosmica as C
from paper_2502_06319_amd import scan as S

pytestmark = pytest.mark.gpu

LNP0, DLNP, NK = math.log(0.05), 0.25, 40


def _tables():
    lnP = LNP0 + DLNP * np.arange(NK)
    rows = [math.log(1.9e4) - g * lnP for g in np.linspace(2.3, 3.3, 16)]
    for kb in (10, 18, 26):  # broken power laws, break on a knot
        b = LNP0 + DLNP * kb
        rows.append(np.where(lnP < b, 9.9 - 2.6 * lnP, 9.9 - 2.6 * b - 3.2 * (lnP - b)))
    for c in (0.05, 0.1, 0.2, 0.3, 0.4):  # curved in log-log
        rows.append(9.5 - 2.7 * lnP - c * (lnP - 1.0) ** 2)
    return np.array(rows)


def test_radial_fp64_reweighting_equals_the_oracle(eng, orc, W, othreads):
    job = W.c1_job(particles_per_bin=512)
    tabs = _tables()
    plan = eng.plan(job, "fp64")
    plan.execute()
    plan.read()
    g, gse = plan.reweight(LNP0, DLNP, tabs)
    plan.destroy()
    p = orc.params(job)
    for b, r in enumerate(orc.run_job(job, threads=othreads)):
        f, se = orc.reweight_bin(p, r["P0"], r["records"], LNP0, DLNP, tabs)
        np.testing.assert_allclose(g[:, b], f, rtol=1e-12)
        np.testing.assert_allclose(gse[:, b], se, rtol=1e-9)


def test_energy_form_reweighting_equals_the_oracle(eng, orc, W, othreads):
    job = W.c2_job(particles_per_bin=300, n_bins=5)
    job["formulation"] = 1
    job["helio"]["hcs"] = 0
    tabs = _tables()[::4]
    plan = eng.plan(job, "fp64")
    plan.execute()
    plan.read()
    g, _ = plan.reweight(LNP0, DLNP, tabs)
    plan.destroy()
    p = orc.params(job)
    for b, r in enumerate(orc.run_job(job, threads=othreads)):
        f, _ = orc.reweight_bin(p, r["P0"], r["records"], LNP0, DLNP, tabs)
        np.testing.assert_allclose(g[:, b], f, rtol=1e-6)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("formulation", [0, 1])
def test_own_power_law_reproduces_the_plan(eng, W, precision, formulation):
    jobs = [W.c2_job(particles_per_bin=400, n_bins=5), W.c1_job(particles_per_bin=200)]
    jobs[1]["job_tag"] = 3
    jobs[0]["formulation"] = formulation
    plan = eng.plan(jobs, precision)
    plan.execute()
    res = plan.read()
    sp = jobs[0]["species"]  # both jobs carry the same proton spectrum
    lnJ, lnP0, dlnP = S.power_law_tables([sp["lis_norm"]], [sp["lis_index"]])
    g, gse = plan.reweight(lnP0, dlnP, lnJ)
    many, _ = plan.reweight(lnP0, dlnP, np.repeat(lnJ, 37, axis=0))  # three groups of 16
    plan.destroy()
    flux = np.concatenate([r["flux"] for r in res])
    se = np.concatenate([r["flux_se"] for r in res])
    np.testing.assert_allclose(g[0], flux, rtol=1e-12)
    np.testing.assert_allclose(gse[0], se, rtol=1e-9)
    for row in many:
        np.testing.assert_array_equal(row, g[0])


def test_reweight_rejects_bad_calls(eng, W):
    plan = eng.plan(W.c1_job(particles_per_bin=16), "mixed")
    lnJ, lnP0, dlnP = S.power_law_tables([1.9e4], [2.78])
    with pytest.raises(C.CosmicaError):
        plan.reweight(lnP0, dlnP, lnJ)  # not executed yet
    plan.execute()
    with pytest.raises(C.CosmicaError):
        plan.reweight(lnP0, -1.0, lnJ)
    with pytest.raises(C.CosmicaError):
        plan.reweight(lnP0, dlnP, np.zeros((1, 1)))
    bad = lnJ.copy()
    bad[0, 3] = np.nan
    with pytest.raises(C.CosmicaError):
        plan.reweight(lnP0, dlnP, bad)
    # the limits: spectra per call and knots per table
    many = np.zeros((C.MAX_REWEIGHT + 1, 2))
    with pytest.raises(C.CosmicaError):
        plan.reweight(lnP0, dlnP, many)
    plan.reweight(lnP0, dlnP, many[:C.MAX_REWEIGHT])
    with pytest.raises(C.CosmicaError):
        plan.reweight(lnP0, dlnP, np.zeros((1, C.MAX_LIS_KNOTS + 1)))
    f, _ = plan.reweight(lnP0, dlnP, np.zeros((1, C.MAX_LIS_KNOTS)))  # J = 1 everywhere
    assert np.all(f > 0)
    plan.destroy()


def test_scan_recovers_the_parameters_of_an_observation(eng, W):
    base = W.c2_job(particles_per_bin=2000, n_bins=8)
    truth = dict(base, seed=777)
    truth["helio"] = S._apply(base["helio"], {"kappa0_scale": 1.3})
    truth["species"] = dict(base["species"], lis_index=2.9)
    obs = eng.run(truth, "mixed")[0]
    err = np.maximum(obs["flux_se"], 0.01 * obs["flux"])
    indices = [2.6, 2.78, 2.9, 3.0, 3.2]
    tabs = S.power_law_tables([base["species"]["lis_norm"]], indices)
    res = S.scan(eng, base, {"kappa0_scale": [0.8, 1.0, 1.3, 1.6, 2.0]}, tabs, "mixed")
    out = S.fit(res, obs["flux"], err, lis_params=np.array(indices)[:, None])
    print("scan fit:", out["best_point"], indices[out["best_lis"]], out["mean"], out["sd"],
          out["chi2_min"], flush=True)
    assert out["best_point"]["kappa0_scale"] == 1.3
    assert indices[out["best_lis"]] == 2.9
    assert abs(out["mean"]["kappa0_scale"] - 1.3) < 0.1
    assert abs(out["mean"]["lis"][0] - 2.9) < 0.05
