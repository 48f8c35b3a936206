"""Register, scratch and occupancy properties of the block kernels, read from
the gfx950 code object metadata that hipcc emits (no GPU needed).

These are the properties the selection loop's speed rests on: the 4-wave FP64
kernel fits five blocks per CU (at most 96 VGPRs), and no kernel keeps the
step's arrays in scratch memory (a step kept out of line puts them there; the
FP32 loops once ran 1.5x slower that way)."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2207_00238_amd import build

HIPCC = build.HIPCC
SRC = os.path.join(build.CSRC, "fse_kernels.hip")

pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which(HIPCC)), reason="hipcc not available")


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    out = tmp_path_factory.mktemp("asm") / "fse_kernels.s"
    flags = [f for f in build.FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [HIPCC] + flags + ["--cuda-device-only", "-S", SRC, "-o", str(out)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-2000:]
    text = open(out).read()
    meta = {}
    # one metadata record per kernel: .name, then its fields (in alphabetical
    # order) up to .wavefront_size
    for m in re.finditer(r"\.name:\s+(_ZN3fse12k_fse_blocksILi(\d+)ELi(\d+)ELb([01])EEEvNS_10LaunchArgsEi)\b(.*?)"
                         r"\.wavefront_size:", text, re.S):
        nw, prec, wide, body = int(m.group(2)), int(m.group(3)), int(m.group(4)), m.group(5)

        def field(name):
            f = re.search(r"\." + name + r":\s+(\d+)", body)
            return int(f.group(1)) if f else None

        meta[(nw, prec, wide)] = {"vgpr": field("vgpr_count"), "scratch": field("private_segment_fixed_size"),
                                  "spill": field("vgpr_spill_count")}
    return meta


def test_every_instance_is_found(kernels):
    expected = {(nw, p, 0) for nw in (1, 2, 4) for p in (0, 1, 2)} | {(8, p, 1) for p in (0, 1, 2)}
    assert expected <= set(kernels), sorted(kernels)


def test_four_wave_fp64_kernel_fits_five_blocks_per_cu(kernels):
    # 512 VGPRs per SIMD lane: five waves need at most 102, allocated in steps of 8
    assert kernels[(4, 0, 0)]["vgpr"] <= 96, kernels[(4, 0, 0)]


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("nw", [1, 2, 4])
def test_reduced_precision_kernels_use_no_scratch(kernels, nw, prec):
    assert kernels[(nw, prec, 0)]["scratch"] == 0, kernels[(nw, prec, 0)]


def test_fp64_kernels_scratch_is_register_spills_only(kernels):
    # the 32 x 32 FP64 kernels spill a few per-workgroup constants at most;
    # arrays of a step kept in scratch would take far more
    for nw in (1, 2, 4):
        k = kernels[(nw, 0, 0)]
        assert k["scratch"] <= 4 * (k["spill"] or 0) + 16, (nw, k)
