"""Pins of the oracle's random numbers (Sec. IV.A: Philox4x32-10, one
Wiener increment sqrt(ds) N(0,1) per step, Sec. III).

* The oracle's Philox4x32-10 is checked bit for bit against an independent
  implementation: rocRAND's header-only engine compiled for and run on the
  host (tests/philox_rocrand_ref.cpp).
* The Box-Muller normals are checked against the standard normal law:
  moments and a Kolmogorov-Smirnov test (scipy).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "philox_rocrand_ref.cpp")])
    return exe


def _counters(rng, n):
    seeds = rng.integers(0, 2**64, n, dtype=np.uint64)
    ctr = rng.integers(0, 2**32, (n, 4), dtype=np.uint64)
    # edge words: all-zero and all-ones counters and keys
    seeds[0], ctr[0] = 0, 0
    seeds[1], ctr[1] = 2**64 - 1, 2**32 - 1
    seeds[2], ctr[2] = 42, [0, 1, 2, 3]
    return seeds, ctr


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(7)
    seeds, ctr = _counters(rng, 4000)
    lines = "\n".join(f"{int(s)} {' '.join(str(int(c)) for c in cc)}" for s, cc in zip(seeds, ctr))
    out = subprocess.run([rocrand_ref], input=lines, capture_output=True, text=True, check=True)
    ref = np.array([[int(x) for x in ln.split()] for ln in out.stdout.strip().splitlines()],
                   dtype=np.uint64)
    got = np.array([orc.philox(int(s), cc) for s, cc in zip(seeds, ctr)], dtype=np.uint64)
    assert ref.shape == got.shape == (4000, 4)
    np.testing.assert_array_equal(got, ref)


def test_philox_counter_words_all_matter(orc):
    base = orc.philox(42, [5, 6, 7, 8])
    for w in range(4):
        c = [5, 6, 7, 8]
        c[w] ^= 1
        assert not np.array_equal(orc.philox(42, c), base)
    assert not np.array_equal(orc.philox(43, [5, 6, 7, 8]), base)
    assert not np.array_equal(orc.philox(42 + (1 << 32), [5, 6, 7, 8]), base)


def test_normals_are_standard(orc):
    n = 50_000
    z = np.array([orc.normals(42, [i, 3, 1, 0]) for i in range(n)]).reshape(-1)
    m = z.size
    assert abs(z.mean()) < 5 / np.sqrt(m)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / m)
    kurt = stats.kurtosis(z, fisher=True)
    assert abs(kurt) < 5 * np.sqrt(24.0 / m)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # the two members of each Box-Muller pair are uncorrelated
    zz = z.reshape(-1, 4)
    for a, b in ((0, 1), (2, 3), (0, 2), (1, 3)):
        assert abs(np.corrcoef(zz[:, a], zz[:, b])[0, 1]) < 5 / np.sqrt(n)
    # largest magnitude: uniforms live in [2^-24, 1 - 2^-24]
    assert np.abs(z).max() <= np.sqrt(-2 * np.log(2.0**-24)) + 1e-12


def test_rng_block_is_the_single_call_loop(orc):
    w, z = orc.rng_block(99, 5, 6, 7, 8, 300)
    for i in (0, 1, 17, 299):
        np.testing.assert_array_equal(w[i], orc.philox(99, [5 + i, 6, 7, 8]))
        np.testing.assert_array_equal(z[i], orc.normals(99, [5 + i, 6, 7, 8]))
