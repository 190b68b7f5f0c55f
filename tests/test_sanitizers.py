"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (plain C) built with both sanitizers runs every entry point on
  small 1D and 3D inputs: momentum and energy forms, heliosheath, orbit,
  capped particles, reduction, re-weighting, the range histogram, a
  checkpoint step and a rejected parameter set.
* The library's host code (runtime.cpp; each sanitizer flag passed to the
  host compiler only, the device code as built) runs job validation,
  error strings, NULL handles and a context on a missing device.
Any report fails the run (no recovery, leak detection on).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe):
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=ENV)
    assert out.returncode == 0, (out.stdout[-2000:], out.stderr[-4000:])
    return out.stdout


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "oracle_driver"
    subprocess.run([gcc, "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-fopenmp",
                    "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "cosmica_oracle.c"),
                    os.path.join(HERE, "oracle_driver.c"), "-lm", "-o", str(exe)],
                   check=True, capture_output=True, timeout=300)
    assert "oracle ok" in _run(exe)


def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    gcc = shutil.which("gcc")
    if not os.path.exists(hipcc) or gcc is None:
        pytest.skip("hipcc or gcc not available")
    csrc = os.path.join(ROOT, "paper_2502_06319_amd", "csrc")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all"]
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I",
              os.path.join(ROOT, "include"), "-I", csrc, "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops", '-DCOSMICA_KERNEL_ID="sanitize"']
    rt, kn, dr = tmp_path / "rt.o", tmp_path / "k.o", tmp_path / "d.o"
    subprocess.run([hipcc] + common + host_san + ["-x", "hip", "-c", os.path.join(csrc, "runtime.cpp"),
                    "-o", str(rt)], check=True, capture_output=True, timeout=600)
    subprocess.run([hipcc] + common + ["-c", os.path.join(csrc, "kernels.hip"), "-o", str(kn)],
                   check=True, capture_output=True, timeout=600)
    subprocess.run([gcc, "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-I",
                    os.path.join(ROOT, "include"), "-c", os.path.join(HERE, "library_driver.c"),
                    "-o", str(dr)], check=True, capture_output=True, timeout=300)
    exe = tmp_path / "library_driver"
    subprocess.run([hipcc, "--offload-arch=gfx950"] + host_san + [str(dr), str(rt), str(kn),
                    "-lpthread", "-o", str(exe)], check=True, capture_output=True, timeout=300)
    assert "library host code ok" in _run(exe)
