"""Register and scratch use of every kernel in the built library, read from the
gfx950 code objects' metadata (no GPU needed).

A kernel that reaches a small table in its arguments through a run-time
index or pointer gets the table copied to scratch memory for every lane.
That cost the split viscous face kernel 3.6x and the fused boundary variants
3.4-4.5x before it was found. A register count one above 256 halves a
kernel's occupancy. Both show only in the timings, so they are checked here
on the build itself."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2306_14011_amd", "libfv.so")
LLVM = "/opt/rocm/llvm/bin"
TOOLS = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"

pytestmark = pytest.mark.skipif(not os.path.exists(LIB) or not all(os.path.exists(t) for t in TOOLS),
                                reason="needs the built library and the ROCm LLVM tools")


def waves_per_simd(regs):
    """Wavefronts a SIMD holds for a kernel of `regs` registers per lane
    (VGPRs and AGPRs together): 512 per lane, allocated in blocks of 8."""
    blocks = (max(regs, 1) + 7) // 8 * 8
    return min(8, 512 // blocks)


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    d = tmp_path_factory.mktemp("codeobj")
    fat = d / "fatbin"
    subprocess.run([TOOLS[0], f"--dump-section=.hip_fatbin={fat}", LIB, str(d / "lib.so")], check=True,
                   capture_output=True)
    data = fat.read_bytes()
    starts = []
    i = data.find(MAGIC)
    while i >= 0:
        starts.append(i)
        i = data.find(MAGIC, i + 1)
    starts.append(len(data))
    out = {}
    for k in range(len(starts) - 1):
        b = d / f"bundle{k}"
        co = d / f"co{k}"
        b.write_bytes(data[starts[k]:starts[k + 1]])
        subprocess.run([TOOLS[1], "--unbundle", "--type=o", f"--targets={TARGET}", f"--input={b}", f"--output={co}"],
                       check=True, capture_output=True)
        notes = subprocess.run([TOOLS[2], "--notes", str(co)], check=True, capture_output=True, text=True).stdout
        for blk in notes.split("\n  - ")[1:]:
            fields = {}
            for line in blk.splitlines():
                line = line.strip().lstrip("- ")
                if ":" in line:
                    key, _, val = line.partition(":")
                    fields.setdefault(key.strip(), val.strip())
            if ".name" in fields and ".vgpr_count" in fields:
                out[fields[".name"]] = {"vgpr": int(fields[".vgpr_count"]),
                                        "private": int(fields[".private_segment_fixed_size"])}
    shutil.rmtree(d, ignore_errors=True)
    return out


def test_every_source_has_kernels(kernels):
    assert len(kernels) >= 100
    for stem in ("k_fused2d", "k_fused3d", "k_adj_stage", "k_visc", "k_flux", "k_sweep_mfma", "k_train"):
        assert any(stem in n for n in kernels), stem


def test_no_kernel_uses_scratch(kernels):
    bad = {n: k["private"] for n, k in kernels.items() if k["private"] != 0}
    assert not bad, bad


def test_every_kernel_runs_two_waves_per_simd(kernels):
    bad = {n: k["vgpr"] for n, k in kernels.items() if waves_per_simd(k["vgpr"]) < 2}
    assert not bad, bad


def test_headline_stage_kernels_run_three_waves_per_simd(kernels):
    # the periodic / transmissive 2D stage kernels without a source term
    # (k_fused2d<STAGE, false, 0>), the curvilinear stage-1 kernel without a
    # source (k_fused2d<0, false, 3>, which asks for three waves) and the
    # matrix-core sweep
    names = [n for n in kernels if "k_fused2dILi" in n and "ELb0ELi0EE" in n] + \
            [n for n in kernels if "k_fused2dILi0ELb0ELi3EE" in n] + \
            [n for n in kernels if "k_sweep_mfma" in n]
    assert len(names) >= 5
    for n in names:
        assert waves_per_simd(kernels[n]["vgpr"]) >= 3, (n, kernels[n]["vgpr"])


def test_waves_per_simd_rule():
    assert waves_per_simd(128) == 4 and waves_per_simd(168) == 3 and waves_per_simd(170) == 2
    assert waves_per_simd(256) == 2 and waves_per_simd(257) == 1 and waves_per_simd(24) == 8
