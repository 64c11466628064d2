"""Machine-code checks of the gfx950 kernels (compiled here, no GPU).

Every DPP row_newbcast broadcast must be a standalone v_mov_b32_dpp: folded
into other VOP2 instructions it produced wrong results on gfx950.  The kernels
must not spill to scratch, and GPU code must not store through the scalar data
cache.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2008_10273_amd", "csrc")
# Sources with the per-file flags the build passes.
SOURCES = [("pdinp_kernels.hip", []),
           ("pdinp_wide.hip", ["-mllvm", "-pragma-unroll-threshold=1000000"]),
           ("pdinp_diffusion.hip", []),
           ("pdinp_select.hip", [])]


@pytest.fixture(scope="module")
def isa(tmp_path_factory):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("isa")
    text = []
    for name, extra in SOURCES:
        out = d / (name + ".s")
        subprocess.check_call([hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                               "-Xclang", "-packed-fp32-ops", *extra, "-I", os.path.join(ROOT, "include"),
                               "--cuda-device-only", "-S", os.path.join(CSRC, name), "-o", str(out)],
                              stderr=subprocess.DEVNULL)
        text.append(out.read_text())
    return "\n".join(text)


def test_newbcast_only_in_standalone_moves(isa):
    dpp = [l.split()[0] for l in isa.splitlines() if "row_newbcast" in l]
    assert dpp, "no broadcasts found"
    assert set(dpp) == {"v_mov_b32_dpp"}, sorted(set(dpp))


def test_no_scratch_spills(isa):
    """No kernel reads or writes scratch memory (register spills or private
    arrays); a few bytes of reserved but unused frame are tolerated."""
    sizes = [int(x) for x in re.findall(r"\.amdhsa_private_segment_fixed_size\s+(\d+)", isa)]
    assert sizes and max(sizes) <= 64, sizes
    used = [l for l in isa.splitlines() if re.match(r"\s*(scratch_|buffer_(load|store))", l)]
    assert not used, used[:5]
    spills = [int(x) for x in re.findall(r"\.vgpr_spill_count:\s+(\d+)", isa)]
    assert spills and max(spills) == 0, spills


def test_no_scalar_stores(isa):
    bad = [l for l in isa.splitlines() if re.match(r"\s*s_(store|atomic|buffer_store|dcache_wb)", l)]
    assert not bad, bad[:5]
