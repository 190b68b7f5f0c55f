"""Whole-path parity of the HIP library against the FP64 oracle (C ABI).

Each run integrates every particle to the boundary (Sec. III, Eq.(3)), then
bins and LIS-weights the exit rigidities (Eq.(4), J = f P^2, L = 0).  Both
sides use the same Philox streams, so comparisons are particle by particle
wherever the arithmetic allows:

* radial model, FP64: every particle takes the same number of steps; exit
  rigidities agree to 1e-12; histograms are identical; flux to 1e-12.
* 3D model, FP64: last-bit differences (FMA contraction, libm vs ocml) flip
  rare threshold decisions -- current-sheet crossings, the slow/fast wind
  band, the exit step -- after which a path continues on other random
  numbers; at least 75 % of the particles of every bin (90 % overall) take
  identical step counts, and each bin's flux is within half a standard error.
* mixed precision: binary32 rounding flips threshold decisions much more
  often, and paths that ride the thin current sheet for 10^4 steps decorrelate
  completely; the GPU and the oracle are then two Monte Carlo estimates on
  partly shared random numbers.  The stated per-bin tolerance is the paired
  one: with w = J_LIS(P_ex)/P_ex^2 per particle on both sides,
      |J_gpu - J_oracle| <= 4 SE_pair,   SE_pair = P0^2 sd(w_gpu - w_orc) / sqrt(N),
  i.e. the mixed path is unbiased against the FP64 oracle at four standard
  errors of the paired difference (SE_pair -> 0 where paths coincide, ->
  sqrt(2) SE where they decorrelate).  Where paths stay correlated (the
  config-3 workload) every bin also lies inside one standard error or the
  paper's 1/sqrt(N) band of Sec. VIII.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2502_06319_amd import cosmica as C

pytestmark = pytest.mark.gpu


def _weights(P, norm=1.9e4, index=2.78):
    return norm * P ** (-index) / (P * P)


def _split(job, exits):
    out, off = [], 0
    for n in job["particles_per_bin"]:
        out.append(exits[off:off + n])
        off += n
    return out


def _contributions(ex, P0, job=None):
    """Each exit's contribution to J_mod(P0): P0^2 J_LIS(P_ex)/P_ex^2 in the
    momentum form; beta0/beta_ex J_LIS(P_ex) exp(-loss) in the energy form."""
    if job is None or job.get("formulation", 0) == 0:
        return P0 * P0 * _weights(ex["P"])
    sp = job["species"]
    Z, M = abs(sp["charge"]), sp["mass_gev"]
    beta = lambda P: Z * P / np.sqrt((Z * P) ** 2 + M * M)
    return beta(P0) / beta(ex["P"]) * sp["lis_norm"] * ex["P"] ** (-sp["lis_index"]) * np.exp(
        -ex["loss"])


def _paired(ge, oe, P0, job=None):
    d = _contributions(ge, P0, job) - _contributions(oe, P0, job)
    N = len(d)
    dJ = d.mean()
    se_pair = d.std(ddof=1) / math.sqrt(N) if N > 1 else 0.0
    return dJ, se_pair


def _report(tag, b, res_o, g_flux, same, dJ, se_pair):
    print(f"{tag} bin {b} P0 {res_o['P0']:.3f}: same_n {same:.4f} dJ/J {dJ / res_o['flux']:+.2e} "
          f"dJ/SE {dJ / res_o['flux_se']:+.3f} dJ/SEpair {dJ / se_pair if se_pair else 0:+.2f}",
          flush=True)


def test_radial_fp64_particle_by_particle(eng, orc, W, othreads):
    job = W.c1_job()
    g = eng.run(job, precision="fp64", exits=True)[0]
    o = orc.run_job(job, threads=othreads)
    for b, (ge, r) in enumerate(zip(_split(job, g["exits"]), o)):
        oe = r["records"]
        np.testing.assert_array_equal(ge["n"], oe["n"])
        np.testing.assert_allclose(ge["P"], oe["P"], rtol=1e-12)
        np.testing.assert_allclose(ge["t"], oe["t"], rtol=1e-12)
        np.testing.assert_allclose(ge["r"], oe["r"], rtol=1e-12)
        np.testing.assert_array_equal(g["hist"][b], r["hist"])
        assert g["steps"][b] == r["steps"]
        assert g["flux"][b] == pytest.approx(r["flux"], rel=1e-12)
        assert g["flux_se"][b] == pytest.approx(r["flux_se"], rel=1e-9)
        assert g["mean_exit_time_s"][b] == pytest.approx(r["mean_exit_time_s"], rel=1e-12)
        assert g["n_capped"][b] == 0 and g["n_nan"][b] == 0


def test_radial_mixed(eng, orc, W, othreads):
    job = W.c1_job()
    g = eng.run(job, precision="mixed", exits=True)[0]
    o = orc.run_job(job, threads=othreads)
    for b, (ge, r) in enumerate(zip(_split(job, g["exits"]), o)):
        same = np.mean(ge["n"] == r["records"]["n"])
        assert same >= 0.99
        assert abs(g["flux"][b] / r["flux"] - 1.0) <= 1e-4
        assert abs(int(g["steps"][b]) - int(r["steps"])) <= 1e-3 * r["steps"]


_ORACLE = {}


def _oracle_run(orc, job, othreads):
    """The oracle's results for a job, computed once per test session (the FP64
    and mixed comparisons of a workload share them)."""
    key = json.dumps(job, sort_keys=True)
    if key not in _ORACLE:
        _ORACLE[key] = orc.run_job(job, threads=othreads)
    return _ORACLE[key]


def _compare_3d(eng, orc, job, precision, othreads, tag):
    g = eng.run(job, precision=precision, exits=True)[0]
    o = _oracle_run(orc, job, othreads)
    tot_same = 0
    stats = []
    for b, (ge, r) in enumerate(zip(_split(job, g["exits"]), o)):
        oe = r["records"]
        N = len(oe)
        same = np.mean(ge["n"] == oe["n"])
        tot_same += same * N
        dJ, se_pair = _paired(ge, oe, r["P0"], job)
        assert dJ == pytest.approx(g["flux"][b] - r["flux"], rel=1e-6, abs=1e-12 * r["flux"])
        _report(tag, b, r, g["flux"][b], same, dJ, se_pair)
        assert int(g["hist"][b].sum()) == N
        assert g["n_nan"][b] == 0 and g["n_capped"][b] == 0
        stats.append((same, dJ, se_pair, r, g["flux_se"][b]))
    return tot_same / sum(job["particles_per_bin"]), stats


def _c2_variant(W, which, n):
    """The config-2 heliosphere with protons at A > 0 (qA > 0, the config
    itself), protons at A < 0, or electrons at A > 0: the last two drift the
    other way (sign of Z times A in Eq.(3)'s drift) and ride the current sheet."""
    job = W.c2_job(particles_per_bin=n)
    if which == "p_A-":
        job["helio"]["polarity"] = -1
    elif which == "e_A+":
        job["species"] = W.species("e-")
    return job


def _unbiased_gates(stats, tag):
    """Sheet-riding paths decorrelate between two implementations (rounding
    changes sheet crossings, Sec. VIII's statistical agreement is the bar):
    per bin |dJ| <= 4 SE_pair, and over the k bins the mean of
    dJ / sqrt(SE_o^2 + SE_g^2) within 3 / sqrt(k) of zero, so a common bias of
    a fraction of the bins' standard errors fails even where each bin passes."""
    z = []
    for same, dJ, se_pair, r, se_g in stats:
        assert abs(dJ) <= 4.0 * se_pair + 1e-12 * r["flux"]
        z.append(dJ / math.hypot(r["flux_se"], se_g))
    z = np.array(z)
    print(f"{tag}: {len(z)} bins, mean dJ/SE_comb {z.mean():+.3f} (gate {3 / math.sqrt(len(z)):.3f}),"
          f" largest |dJ/SE_comb| {np.abs(z).max():.2f}", flush=True)
    assert abs(z.mean()) <= 3.0 / math.sqrt(len(z))


@pytest.mark.parametrize("which", ["p_A+", "p_A-", "e_A+"])
def test_3d_fp64_against_oracle(eng, orc, W, othreads, which):
    """Config 2 (20 bins x 5,000 protons, qA > 0) and the drift-reversed
    populations at 2,000 per bin."""
    job = _c2_variant(W, which, 5000 if which == "p_A+" else 2000)
    overall, stats = _compare_3d(eng, orc, job, "fp64", othreads, f"3d-fp64 {which}")
    print(f"3d-fp64 {which}: identical step counts overall {overall:.4f}", flush=True)
    if which == "p_A+":
        assert overall >= 0.90
        for same, dJ, se_pair, r, se_g in stats:
            assert same >= 0.75
            assert abs(dJ) <= 0.5 * r["flux_se"]
            assert abs(dJ) <= 4.0 * se_pair + 1e-12 * r["flux"]
    else:
        _unbiased_gates(stats, f"3d-fp64 {which}")


@pytest.mark.parametrize("which", ["p_A+", "p_A-", "e_A+"])
def test_3d_mixed_against_oracle(eng, orc, W, othreads, which):
    """The mixed-precision form (FP32 bulk, FP64 r, t, P).  Config 3 itself
    (qA > 0, 20 x 5,000): paths stay correlated, and every bin whose paths
    mostly coincide lies within one standard error of the oracle (the 1/sqrt(N)
    band of Sec. VIII), the rest within it or the paired 4 sigma.  The
    drift-reversed populations (2,000 per bin): the unbiasedness gates."""
    job = _c2_variant(W, which, 5000 if which == "p_A+" else 2000)
    overall, stats = _compare_3d(eng, orc, job, "mixed", othreads, f"3d-mixed {which}")
    print(f"3d-mixed {which}: identical step counts overall {overall:.4f}", flush=True)
    if which == "p_A+":
        assert overall >= 0.2
        for same, dJ, se_pair, r, se_g in stats:
            N = r["n_used"]
            assert abs(dJ) <= 4.0 * se_pair + 1e-12 * r["flux"]
            if same >= 0.5:
                assert abs(dJ) <= r["flux_se"]
            else:
                assert abs(dJ) <= max(r["flux_se"], r["flux"] / math.sqrt(N))
    else:
        _unbiased_gates(stats, f"3d-mixed {which}")


def test_batched_sheet_riding_bins_unbiased(eng, orc, W, othreads):
    """Mixed precision against the oracle on 16 drift-reversed (qA < 0) bins of
    the batched workload with 5,000-8,000 particles each, four per species:
    these particles ride the current sheet for 10^4-10^5 steps and carry most
    of the batched workload's steps.  Each bin runs on its own Philox streams
    (bin_offset), as inside the batch."""
    jobs = W.c4_jobs()
    cands = {}
    for ji, j in enumerate(jobs):
        if np.sign(j["species"]["charge"]) * j["helio"]["polarity"] > 0:
            continue
        for b, n in enumerate(j["particles_per_bin"]):
            if 5000 <= n <= 8000:
                cands.setdefault(j["species"]["name"], []).append((ji, b))
    rng = np.random.default_rng(7)
    picked = []
    for sp in ("p", "He4", "He3", "e-"):
        picked += [cands[sp][i] for i in rng.choice(len(cands[sp]), 4, replace=False)]
    subs = [dict(jobs[ji], rigidity_gv=[jobs[ji]["rigidity_gv"][b]],
                 particles_per_bin=[jobs[ji]["particles_per_bin"][b]], bin_offset=b)
            for ji, b in picked]
    gres = eng.run(subs, precision="mixed", exits=True)
    stats = []
    for (ji, b), sub, g in zip(picked, subs, gres):
        r = orc.run_job(sub, threads=othreads)[0]
        dJ, se_pair = _paired(g["exits"], r["records"], r["P0"])
        assert dJ == pytest.approx(g["flux"][0] - r["flux"], rel=1e-6, abs=1e-12 * r["flux"])
        _report(f"batched sheet-riding job {ji} {sub['species']['name']} N {r['n_used']}", b, r,
                g["flux"][0], np.mean(g["exits"]["n"] == r["records"]["n"]), dJ, se_pair)
        print(f"  mean steps gpu {g['steps'][0] / r['n_used']:.0f} oracle "
              f"{r['steps'] / r['n_used']:.0f}; SE/J oracle {r['flux_se'] / r['flux']:.3f} gpu "
              f"{g['flux_se'][0] / g['flux'][0]:.3f}", flush=True)
        assert g["n_nan"][0] == 0 and g["n_capped"][0] == 0
        stats.append((0.0, dJ, se_pair, r, g["flux_se"][0]))
    _unbiased_gates(stats, "batched sheet-riding bins, mixed")


def test_full_size_3d_fp64_sampled_particles(eng, orc, W, othreads):
    """Config-2 size (20 bins x 5,000): particles 0-63 and 4936-4999 of every bin."""
    job = W.c2_job()
    g = eng.run(job, precision="fp64", exits=True)[0]
    same = []
    for b, ge in enumerate(_split(job, g["exits"])):
        assert int(g["hist"][b].sum()) == 5000 and g["n_nan"][b] == 0
        for first in (0, 4936):
            sub = dict(job, rigidity_gv=[job["rigidity_gv"][b]], particles_per_bin=[64],
                       bin_offset=b)
            oe = orc.run_job(sub, threads=othreads, first=first)[0]["records"]
            gs = ge[first:first + 64]
            m = gs["n"] == oe["n"]
            same.append(m.mean())
            if m.any():
                assert np.median(np.abs(gs["P"][m] / oe["P"][m] - 1.0)) <= 1e-9
    assert np.mean(same) >= 0.85


def test_full_size_batched_mixed(eng, orc, W, othreads):
    """The batched workload at full size (64 sets x 4 species x 30 bins, ~4.0e7
    particles) in the launch shape the benchmark times, first and repeated
    execution: invariants over every bin, and sampled bins against the oracle
    with paired statistics."""
    from bench import tuned_engine_launch

    jobs = W.c4_jobs()
    tuned_engine_launch(eng, {"mixed": jobs})
    plan = eng.plan(jobs, "mixed", exits=True)
    plan.execute()
    res = plan.read(exits=True)
    # the benchmark times repeated executions of one plan: bitwise the same
    # results
    plan.execute()
    again = plan.read(exits=True)
    plan.destroy()
    for a, b in zip(again, res):
        for k in ("hist", "flux", "flux_se", "mean_exit_time_s", "steps", "n_capped", "n_nan"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)
        np.testing.assert_array_equal(a["exits"], b["exits"])
    del again
    total_nan = total_cap = 0
    for j, r in zip(jobs, res):
        N = np.asarray(j["particles_per_bin"])
        np.testing.assert_array_equal(r["hist"].sum(axis=1), N)
        assert np.all(r["steps"] >= N)
        assert np.all(r["exits"]["P"] >= np.repeat(j["rigidity_gv"], N))
        total_nan += int(r["n_nan"].sum())
        total_cap += int(r["n_capped"].sum())
    assert total_nan == 0 and total_cap == 0
    # sampled bins: one of each species, small bins so the oracle finishes quickly
    rng = np.random.default_rng(5)
    picked = []
    for sp in ("p", "He4", "He3", "e-"):
        cands = [(ji, b) for ji, j in enumerate(jobs) if j["species"]["name"] == sp
                 for b, n in enumerate(j["particles_per_bin"]) if n <= 900]
        picked += [cands[i] for i in rng.choice(len(cands), 2, replace=False)]
    for ji, b in picked:
        j = jobs[ji]
        r = orc.run_job(j, threads=othreads, bins=[b])[0]
        ge = _split(j, res[ji]["exits"])[b]
        dJ, se_pair = _paired(ge, r["records"], r["P0"])
        N = r["n_used"]
        _report(f"batched job {ji} {j['species']['name']}", b, r, res[ji]["flux"][b],
                np.mean(ge["n"] == r["records"]["n"]), dJ, se_pair)
        assert abs(dJ) <= 4.0 * se_pair + 1e-12 * r["flux"]
        assert abs(dJ) <= 4.0 * math.hypot(r["flux_se"], res[ji]["flux_se"][b])
