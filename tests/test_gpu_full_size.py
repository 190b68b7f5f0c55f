"""The benchmark's other full-size workloads in the launch shape it times:
the batched workload in nose-squashed heliospheres with a heliosheath, seen
from a moving detection point, and in the energy form (4.0e7 particles each).
For each: invariants over every bin, a second execution (as in the timed
passes) bitwise equal to the first, and
sampled bins against the oracle with the paired statistics of the mixed
precision tolerance."""
import math

import numpy as np
import pytest

from tests.test_gpu_path import _paired, _report, _split

pytestmark = pytest.mark.gpu

KEYS = ("hist", "flux", "flux_se", "mean_exit_time_s", "steps", "n_capped", "n_nan")


def _check(eng, orc, othreads, jobs, tag, n_samples=4, seed=11):
    from bench import tuned_engine_launch

    tuned_engine_launch(eng, {"mixed": jobs})
    plan = eng.plan(jobs, "mixed", exits=True)
    plan.execute()
    res = plan.read(exits=True)
    plan.execute()
    again = plan.read(exits=True)
    plan.destroy()
    for a, b in zip(again, res):
        for k in KEYS:
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)
        np.testing.assert_array_equal(a["exits"], b["exits"])
    del again
    for j, r in zip(jobs, res):
        N = np.asarray(j["particles_per_bin"])
        np.testing.assert_array_equal(r["hist"].sum(axis=1), N)
        assert np.all(r["steps"] >= N)
        assert np.all(r["exits"]["P"] >= np.repeat(j["rigidity_gv"], N))
        assert int(r["n_nan"].sum()) == 0 and int(r["n_capped"].sum()) == 0
    rng = np.random.default_rng(seed)
    cands = [(ji, b) for ji, j in enumerate(jobs) for b, n in enumerate(j["particles_per_bin"])
             if n <= 700]
    for i in rng.choice(len(cands), n_samples, replace=False):
        ji, b = cands[i]
        j = jobs[ji]
        r = orc.run_job(j, threads=othreads, bins=[b])[0]
        ge = _split(j, res[ji]["exits"])[b]
        dJ, se_pair = _paired(ge, r["records"], r["P0"], j)
        _report(f"{tag} job {ji} {j['species']['name']}", b, r, res[ji]["flux"][b],
                np.mean(ge["n"] == r["records"]["n"]), dJ, se_pair)
        assert abs(dJ) <= 4.0 * se_pair + 1e-12 * r["flux"]
        assert abs(dJ) <= 4.0 * math.hypot(r["flux_se"], res[ji]["flux_se"][b])


def test_full_size_heliosheath(eng, orc, W, othreads):
    _check(eng, orc, othreads, W.c4_heliosheath_jobs(), "heliosheath")


def test_full_size_orbit(eng, orc, W, othreads):
    _check(eng, orc, othreads, W.c4_orbit_jobs(), "orbit")


def test_full_size_energy_form(eng, orc, W, othreads):
    _check(eng, orc, othreads, [dict(j, formulation=1) for j in W.c4_jobs()], "energy")
