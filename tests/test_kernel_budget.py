"""Register and scratch budget of the gfx950 kernels, read from the code-object
metadata of a device-only compile (no GPU needed).

The step loop keeps the particle state and the job constants in VGPRs, so a
spill to scratch or a register count past an occupancy step shows up in
throughput at once.  The budget: no kernel spills; the binary32 3D
propagation kernels whose launch shares one Philox key (the batched path)
stay at or below 102 VGPRs (5 waves per SIMD of 512 registers); those with a
key per lane (serving, where each request has its own seed) hold a
scalar-key and a per-lane-key copy of the step loop and stay at or below 128
(4 waves: measured faster than forcing 5, which costs instructions); the
energy form at or below 128; the radial binary32 kernels at or below 102.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2502_06319_amd", "csrc")


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("budget") / "kernels.s"
    cmd = [hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           '-DCOSMICA_KERNEL_ID="budget"', "--cuda-device-only", "-S",
           os.path.join(CSRC, "kernels.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    meta = out.read_text().split(".amdgpu_metadata", 1)[1]
    found = {}
    for block in meta.split("  - ."):
        name = re.search(r"\.name:\s+(\S+)", block)
        vgpr = re.search(r"\.vgpr_count:\s+(\d+)", block)
        scratch = re.search(r"\.private_segment_fixed_size:\s+(\d+)", block)
        if name and vgpr and scratch:
            found[name.group(1)] = (int(vgpr.group(1)), int(scratch.group(1)))
    return found


def _propagate(kernels, real, model_3d, energy=None, shared_key=None):
    # k_propagate<R, M3D, UKEY, SHAPED, ENERGY>: mangled flags Lb0/Lb1 in that order
    pat = re.compile(r"k_propagateI%sLb%dELb([01])ELb[01]ELb([01])E" % (real, int(model_3d)))
    out = {}
    for name, v in kernels.items():
        m = pat.search(name)
        if (m and (energy is None or int(m.group(2)) == int(energy)) and
                (shared_key is None or int(m.group(1)) == int(shared_key))):
            out[name] = v
    return out


def test_no_kernel_spills(kernels):
    assert len(kernels) >= 20
    for name, (vgpr, scratch) in kernels.items():
        assert scratch == 0, f"{name}: {scratch} B of scratch per lane"


def test_binary32_3d_propagation_keeps_five_waves(kernels):
    k = _propagate(kernels, "f", True, energy=False, shared_key=True)
    assert len(k) == 2
    for name, (vgpr, _) in k.items():
        assert vgpr <= 102, f"{name}: {vgpr} VGPRs (5 waves/SIMD need <= 102)"


def test_binary32_3d_per_lane_key_keeps_four_waves(kernels):
    k = _propagate(kernels, "f", True, energy=False, shared_key=False)
    assert len(k) == 2
    for name, (vgpr, _) in k.items():
        assert vgpr <= 128, f"{name}: {vgpr} VGPRs (4 waves/SIMD need <= 128)"


def test_binary32_energy_form_keeps_four_waves(kernels):
    k = _propagate(kernels, "f", True, energy=True)
    assert len(k) == 4
    for name, (vgpr, _) in k.items():
        assert vgpr <= 128, f"{name}: {vgpr} VGPRs (4 waves/SIMD need <= 128)"


def test_radial_binary32_keeps_five_waves(kernels):
    k = _propagate(kernels, "f", False)
    assert len(k) == 2
    for name, (vgpr, _) in k.items():
        assert vgpr <= 102, name
