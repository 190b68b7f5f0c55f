"""Runtime behaviour of the HIP library through the C ABI.

Scheduling invariance: the Philox counter of every step is (n, particle, bin,
job_tag), so neither the launch shape, the refill chunk, the order of the work
queue, the batch a job is packed into, nor splitting its bins over several jobs
changes a single bit of its results.  Edge cases: ragged and single-particle
bins, both models in one batch, the step cap, plans executed repeatedly and
into torch device buffers, the tuner and its cache, the HBM budget.
"""
import math
import os
import time

import numpy as np
import pytest

from paper_2502_06319_amd import cosmica as C

pytestmark = pytest.mark.gpu

KEYS = ("hist", "flux", "flux_se", "mean_exit_time_s", "steps", "n_capped", "n_nan")


def assert_same(a, b, exits=True):
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    if exits:
        np.testing.assert_array_equal(a["exits"], b["exits"])


@pytest.fixture
def restore_launch(eng):
    saved = {(m, p): eng.get_launch(m, p) for m in (0, 1) for p in ("fp64", "mixed")}
    yield
    for (m, p), c in saved.items():
        eng.set_launch(m, p, **c)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_results_do_not_depend_on_launch_shape(eng, W, precision, restore_launch):
    job = W.c2_job(particles_per_bin=700, n_bins=5)
    ref = None
    for shape in [(256, 0, 256, 0), (64, 1, 1, 1), (128, 2, 1024, 0), (256, 3, 7, 1)]:
        eng.set_launch(C.MODEL_3D, precision, *shape)
        r = eng.run(job, precision, exits=True)[0]
        if ref is None:
            ref = r
        else:
            assert_same(r, ref)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_results_do_not_depend_on_the_batch(eng, W, precision):
    a = W.c2_job(particles_per_bin=400, n_bins=6)
    a["job_tag"] = 7
    b = W.c1_job(particles_per_bin=300)
    b["job_tag"] = 3
    c = W.c4_jobs(n_sets=1, n_bins=8, n_min=100, n_max=600)[2]
    alone = eng.run(a, precision, exits=True)[0]
    mix = eng.run([b, a, c], precision, exits=True)
    assert_same(mix[1], alone)
    assert_same(mix[0], eng.run(b, precision, exits=True)[0])


def test_bins_split_over_jobs_with_bin_offset(eng, W):
    whole = W.c2_job(particles_per_bin=300, n_bins=8)
    r = eng.run(whole, "mixed", exits=True)[0]
    parts = []
    for lo, hi in ((0, 3), (3, 8)):
        j = dict(whole, rigidity_gv=whole["rigidity_gv"][lo:hi],
                 particles_per_bin=whole["particles_per_bin"][lo:hi], bin_offset=lo)
        parts.append(eng.run(j, "mixed", exits=True)[0])
    for k in KEYS:
        np.testing.assert_array_equal(np.concatenate([parts[0][k], parts[1][k]]), r[k])
    np.testing.assert_array_equal(np.concatenate([parts[0]["exits"], parts[1]["exits"]]),
                                  r["exits"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ragged_and_single_particle_bins(eng, orc, W, precision, othreads):
    counts = [1, 2, 63, 64, 65, 257]
    job1 = W.c1_job()
    job1["rigidity_gv"] = job1["rigidity_gv"][:6]
    job1["particles_per_bin"] = counts
    job3 = W.c2_job(n_bins=6)
    job3["particles_per_bin"] = counts
    job3["job_tag"] = 1
    g1, g3 = eng.run([job1, job3], precision, exits=True)
    for g in (g1, g3):
        np.testing.assert_array_equal(g["hist"].sum(axis=1), counts)
        assert np.all(g["exits"]["n"] >= 1)
        assert g["flux_se"][0] == 0.0  # one particle: no spread estimate
    if precision == "fp64":  # radial model, FP64: particle by particle
        o = orc.run_job(job1, threads=othreads)
        np.testing.assert_array_equal(g1["exits"]["n"],
                                      np.concatenate([r["records"]["n"] for r in o]))
        for b, r in enumerate(o):
            np.testing.assert_array_equal(g1["hist"][b], r["hist"])


def test_step_cap(eng, orc, W, othreads):
    job = W.c1_job(particles_per_bin=200)
    job["step_cap"] = 150
    g = eng.run(job, "fp64", exits=True)[0]
    assert eng.last_status == C.ESTEPCAP
    o = orc.run_job(job, threads=othreads)
    for b, r in enumerate(o):
        assert g["n_capped"][b] == r["n_capped"]
        if r["n_used"] > 0:
            assert g["flux"][b] == pytest.approx(r["flux"], rel=1e-12)
    ex = g["exits"]
    assert np.all(ex["n"][ex["flags"] == 1] == 150)
    assert int(sum(g["n_capped"])) == int(np.sum(ex["flags"] == 1)) > 0


def test_plan_repeats(eng, W):
    jobs = [W.c2_job(particles_per_bin=500, n_bins=5), W.c1_job(particles_per_bin=200)]
    jobs[1]["job_tag"] = 9
    plan = eng.plan(jobs, "mixed")
    assert plan.info() == {"bins": 13, "particles": 5 * 500 + 8 * 200, "jobs": 2}
    plan.execute()
    a = plan.read()
    plan.execute()
    b = plan.read()
    for x, y in zip(a, b):
        assert_same(x, y, exits=False)
    plan.destroy()


TORCH_CHILD = r"""
import sys, numpy as np
import torch                                   # first: one HIP runtime for both
sys.path.insert(0, sys.argv[1])
from paper_2502_06319_amd import cosmica as C, workloads as W
jobs = [W.c2_job(particles_per_bin=500, n_bins=5), W.c1_job(particles_per_bin=200)]
jobs[1]["job_tag"] = 9
stream = torch.cuda.Stream()
eng = C.Engine(0, stream=stream)               # runs on torch's stream
for m in (C.MODEL_1D, C.MODEL_3D):             # queue re-sorted after the first execution
    eng.set_launch(m, "mixed", **dict(eng.get_launch(m, "mixed"), order=2))
plan = eng.plan(jobs, "mixed")
plan.execute()
a = plan.read()
nb = 13
dev = torch.device("cuda:0")
out = {"hist": torch.zeros((nb, C.NHIST), dtype=torch.int32, device=dev),
       "flux": torch.zeros(nb, dtype=torch.float64, device=dev),
       "flux_se": torch.zeros(nb, dtype=torch.float64, device=dev),
       "mean_exit_time_s": torch.zeros(nb, dtype=torch.float64, device=dev),
       "steps": torch.zeros(nb, dtype=torch.int64, device=dev),
       "n_capped": torch.zeros(nb, dtype=torch.int32, device=dev),
       "n_nan": torch.zeros(nb, dtype=torch.int32, device=dev)}
torch.cuda.synchronize()
plan.execute(out)
stream.synchronize()
np.testing.assert_array_equal(out["flux"].cpu().numpy(), np.concatenate([a[0]["flux"], a[1]["flux"]]))
np.testing.assert_array_equal(out["hist"].cpu().numpy().astype(np.uint32),
                              np.concatenate([a[0]["hist"], a[1]["hist"]]))
np.testing.assert_array_equal(out["steps"].cpu().numpy().astype(np.uint64),
                              np.concatenate([a[0]["steps"], a[1]["steps"]]))
plan.destroy()
# a plan executed only into device buffers sorts by the counts it wrote there
plan = eng.plan(jobs, "mixed")
for _ in range(2):
    for t in out.values():
        t.zero_()
    torch.cuda.synchronize()
    plan.execute(out)
    stream.synchronize()
    np.testing.assert_array_equal(out["flux"].cpu().numpy(),
                                  np.concatenate([a[0]["flux"], a[1]["flux"]]))
plan.destroy()
eng.close()
print("torch-ok")
"""


def test_torch_stream_and_device_buffers():
    """torch as plumbing: the context runs on a torch stream and a plan writes
    its per-bin results straight into torch device tensors.  Run in a fresh
    process that imports torch first, so that torch and the library share the
    one HIP runtime torch ships with."""
    import subprocess
    import sys

    pytest.importorskip("torch")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", TORCH_CHILD, root], capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert "torch-ok" in out.stdout


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_queue_by_expected_steps_changes_no_bit(eng, W, precision, restore_launch):
    """Queue order 2 starts the bins with the most expected steps per particle
    first (drift-reversed, wavy-sheet bins ahead of the rest): every
    execution's results stay bitwise those of the submission order."""
    jobs = [W.c2_job(particles_per_bin=300, n_bins=6), W.c1_job(particles_per_bin=200),
            W.c4_jobs(n_sets=1, n_bins=8, n_min=50, n_max=400)[3]]
    jobs[1]["job_tag"] = 5
    for m in (C.MODEL_1D, C.MODEL_3D):
        eng.set_launch(m, precision, **dict(eng.get_launch(m, precision), order=0))
    ref = eng.run(jobs, precision, exits=True)
    for m in (C.MODEL_1D, C.MODEL_3D):
        eng.set_launch(m, precision, **dict(eng.get_launch(m, precision), order=2))
    plan = eng.plan(jobs, precision, exits=True)
    for _ in range(3):
        plan.execute()
        for a, b in zip(plan.read(exits=True), ref):
            assert_same(a, b)
    plan.destroy()


def test_plan_job_count_limit(eng, W):
    """More than COSMICA_MAX_JOBS jobs (the kernels address region tables by
    32-bit offsets) is rejected before any job is read."""
    import ctypes

    pack = C._JobPack(W.c1_job(particles_per_bin=4))
    jarr = (C.Job * 1)(pack.job)
    h = ctypes.c_void_p()
    st = C.load().cosmica_plan_create(eng.handle, jarr, C.MAX_JOBS + 1, C.PREC_MIXED, 0,
                                      ctypes.byref(h))
    assert st == C.EINVAL and not h.value


def test_rejected_run_leaves_caller_buffers_untouched(eng, W):
    """cosmica_run validates every job before any device work: on EINVAL the
    caller's result buffers keep what they held."""
    import ctypes

    good = W.c1_job(particles_per_bin=16)
    bad = W.c2_job(particles_per_bin=16, n_bins=4)
    bad["helio"]["kappa0_cm2_s"] = [-1.0] * 15
    packs = [C._JobPack(good), C._JobPack(bad)]
    res = [C._ResultPack(p.n_bins, p.total, True) for p in packs]
    for r in res:
        r.flux[:] = 7.0
        r.hist[:] = 3
        r.exits["P"] = 5.0
    jarr = (C.Job * 2)(*[p.job for p in packs])
    rarr = (C.Result * 2)(*[r.c for r in res])
    st = C.load().cosmica_run(eng.handle, jarr, 2, C.PREC_MIXED, rarr)
    assert st == C.EINVAL
    for r in res:
        assert np.all(r.flux == 7.0) and np.all(r.hist == 3) and np.all(r.exits["P"] == 5.0)


def test_non_finite_particles_are_flagged_and_left_out(eng, W):
    """At 1e20 GV the binary32 square of the rigidity overflows, so the mixed
    path's coefficients are non-finite at the first step: every particle of
    that bin leaves flagged non-finite, is counted, and stays out of the
    histogram and the flux, while the job's other bins are bitwise those of
    the job without it."""
    good = W.c2_job(particles_per_bin=200, n_bins=3)
    bad = dict(good, rigidity_gv=list(good["rigidity_gv"]) + [1e20],
               particles_per_bin=list(good["particles_per_bin"]) + [50])
    a = eng.run(good, "mixed", exits=True)[0]
    b = eng.run(bad, "mixed", exits=True)[0]
    assert b["n_nan"][3] == 50 and b["n_capped"][3] == 0
    assert b["flux"][3] == 0.0 and int(b["hist"][3].sum()) == 0
    ex = b["exits"][-50:]
    assert np.all(ex["flags"] == 2) and np.all(ex["n"] == 1)
    for k in KEYS:
        np.testing.assert_array_equal(b[k][:3], a[k], err_msg=k)
    np.testing.assert_array_equal(b["exits"][:-50], a["exits"])


def test_timings_count_every_step(eng, W):
    job = W.c2_job(particles_per_bin=400, n_bins=4)
    r = eng.run(job, "mixed")[0]
    t = eng.timings()
    assert t["steps"] == int(r["steps"].sum())
    assert t["particles"] == 1600
    assert t["propagate_ms"] > 0 and t["reduce_ms"] > 0
    assert t["grid_blocks"] >= 1 and t["block"] in (64, 128, 256)


def test_tuner_sweeps_once_then_uses_its_cache(W, tmp_path):
    cache = str(tmp_path / "tune.txt")
    with C.Engine(0) as e:
        cfg = e.tune(C.MODEL_1D, "mixed", cache)
        assert cfg["block"] in (64, 128, 256) and cfg["chunk"] >= 1
        line = open(cache).read().split()
        assert len(line) == 8 and float(line[-1]) > 0
        t0 = time.perf_counter()
        cfg2 = e.tune(C.MODEL_1D, "mixed", cache)
        assert time.perf_counter() - t0 < 0.5
        assert cfg2 == cfg
        # tuned shape, identical results
        job = W.c1_job(particles_per_bin=128)
        a = e.run(job, "mixed", exits=True)[0]
        e.set_launch(C.MODEL_1D, "mixed", 256, 0, 256, 0)
        assert_same(e.run(job, "mixed", exits=True)[0], a)


def test_hbm_budget_is_enforced(W):
    with C.Engine(0, hbm_budget_bytes=32 << 20) as e:
        with pytest.raises(C.CosmicaError) as ex:
            e.plan(W.c4_jobs(), "mixed")
        assert ex.value.status == C.ENOMEM
        r = e.run(W.c1_job(particles_per_bin=64), "mixed")[0]  # a small job still fits
        assert int(r["hist"].sum()) == 8 * 64
        # blocks kept for reuse (at most a quarter of the budget: ~7 MB after the
        # first job here) give way to an allocation that needs the room (~27 MB)
        small = W.c2_job(particles_per_bin=17500, n_bins=20)
        big = W.c2_job(particles_per_bin=67500, n_bins=20)
        for job in (small, big, W.c1_job(particles_per_bin=64)):
            r = e.run(job, "mixed")[0]
            assert int(r["hist"].sum()) == int(np.sum(job["particles_per_bin"]))
        assert e.serve_stats()["bytes_in_use"] <= 32 << 20


def test_freed_blocks_are_reused_by_repeated_runs(W):
    """A repeated run of one shape takes its device blocks from the context's
    cache: the bytes held stop growing after the first run, and every run's
    results are bitwise the first's."""
    jobs = [W.c2_job(particles_per_bin=300, n_bins=5), W.c1_job(particles_per_bin=100)]
    with C.Engine(0) as e:
        first = e.run(jobs, "mixed", exits=True)
        held = e.serve_stats()["bytes_in_use"]
        assert held > 0
        for _ in range(4):
            again = e.run(jobs, "mixed", exits=True)
            assert e.serve_stats()["bytes_in_use"] == held
            for a, b in zip(again, first):
                assert_same(a, b)
        plan = e.plan(jobs, "fp64")  # other sizes: new blocks, then reuse
        plan.execute()
        plan.read()
        plan.destroy()
        held64 = e.serve_stats()["bytes_in_use"]
        plan = e.plan(jobs, "fp64")
        plan.execute()
        plan.destroy()
        assert e.serve_stats()["bytes_in_use"] == held64
