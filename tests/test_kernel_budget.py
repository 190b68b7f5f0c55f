"""Register and scratch budget of the gfx950 kernels, read from the code-object
metadata of a device-only compile (no GPU needed).

The step loop keeps the particle state and the job constants in VGPRs, so a
spill to scratch or a register count past an occupancy step shows up in
throughput at once.  Occupancy is the compiler's own figure for each kernel
(waves per SIMD, from its VGPR and SGPR counts and their allocation
granularity).  The budget: no kernel spills; the binary32 3D propagation
kernel for a spherical heliosphere whose launch shares one Philox key (the
batched path) keeps 5 waves per SIMD; every other binary32 3D variant (a
squashed heliosphere, a key per lane for serving, the energy form) keeps 4
(4 waves were measured faster than forcing 5, which costs instructions); the
radial binary32 kernels keep 5.
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
    text = out.read_text()
    code, meta = text.split(".amdgpu_metadata", 1)
    occupancy = {}
    for m in re.finditer(r"\n(_Z\w+):", code):
        occ = re.search(r"; Occupancy: (\d+)", code[m.end():])
        if occ:
            occupancy.setdefault(m.group(1), int(occ.group(1)))
    found = {}
    for block in meta.split("  - ."):
        name = re.search(r"\.name:\s+(\S+)", block)
        vgpr = re.search(r"\.vgpr_count:\s+(\d+)", block)
        scratch = re.search(r"\.private_segment_fixed_size:\s+(\d+)", block)
        if name and vgpr and scratch:
            found[name.group(1)] = (int(vgpr.group(1)), int(scratch.group(1)),
                                    occupancy.get(name.group(1), 0))
    return found


def _propagate(kernels, real, model_3d, energy=None, shared_key=None, shaped=None):
    # k_propagate<R, M3D, UKEY, SHAPED, ENERGY>: mangled flags Lb0/Lb1 in that order
    pat = re.compile(r"k_propagateI%sLb%dELb([01])ELb([01])ELb([01])E" % (real, int(model_3d)))
    out = {}
    for name, v in kernels.items():
        m = pat.search(name)
        if (m and (energy is None or int(m.group(3)) == int(energy)) and
                (shaped is None or int(m.group(2)) == int(shaped)) and
                (shared_key is None or int(m.group(1)) == int(shared_key))):
            out[name] = v
    return out


def test_no_kernel_spills(kernels):
    assert len(kernels) >= 20
    for name, (vgpr, scratch, _) in kernels.items():
        assert scratch == 0, f"{name}: {scratch} B of scratch per lane"


def test_occupancy_is_reported_for_every_propagation_kernel(kernels):
    k = _propagate(kernels, "f", True)
    assert len(k) == 8
    for name, (vgpr, _, occ) in k.items():
        # at least what the VGPR count alone allows (granularity 8 of 512)
        assert 1 <= occ <= min(8, 512 // (-(-vgpr // 8) * 8)), (name, vgpr, occ)


def test_binary32_3d_batched_propagation_keeps_five_waves(kernels):
    k = _propagate(kernels, "f", True, energy=False, shared_key=True, shaped=False)
    assert len(k) == 1
    for name, (vgpr, _, occ) in k.items():
        assert occ >= 5, f"{name}: {vgpr} VGPRs, {occ} waves/SIMD"


def test_binary32_3d_other_variants_keep_four_waves(kernels):
    k = _propagate(kernels, "f", True)
    assert len(k) == 8
    for name, (vgpr, _, occ) in k.items():
        assert occ >= 4, f"{name}: {vgpr} VGPRs, {occ} waves/SIMD"


def test_radial_binary32_keeps_five_waves(kernels):
    k = _propagate(kernels, "f", False)
    assert len(k) == 2
    for name, (vgpr, _, occ) in k.items():
        assert occ >= 5, f"{name}: {vgpr} VGPRs, {occ} waves/SIMD"
