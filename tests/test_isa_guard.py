"""Guard on the generated gfx950 code of the compute kernels (CPU: hipcc
cross-compiles to assembly here).

An address must be formed from the masked neighbour index.  A 64-bit
multiply-add that takes as multiplicand the very register a 24-bit mask was
just taken from has dropped the mask from an address: the code generator
did this for `pos + 24 * (word & 0xffffff)` in the several-species kernels
of the fused packing when the word also carried a row position in its top
bits, and the kernels read positions far out of bounds.  The fused packing
now reads plain indices; this test keeps the pattern out of every kernel."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def dropped_masks(asm: str):
    lines = asm.split("\n")
    kern, hits = None, []
    for i, l in enumerate(lines):
        m = re.match(r"^(_Z\S+):", l)
        if m:
            kern = m.group(1)
        m = re.search(r"v_and_b32_e(?:32|64) (v\d+), 0xffffff, (v\d+)", l)
        if not m:
            continue
        src = m.group(2)
        for j in range(i + 1, min(i + 60, len(lines))):
            t = lines[j].strip()
            if not t or t.startswith((";", ".")):
                continue
            parts = t.split(None, 1)
            if len(parts) < 2:
                continue
            args = [x.strip() for x in parts[1].split(",")]
            if parts[0].startswith(("v_mad_u64_u32", "v_mad_i64_i32")) and src in args[2:4]:
                hits.append((kern, t))
                break
            dst = args[0]
            r = re.fullmatch(r"v\[(\d+):(\d+)\]", dst)
            if dst == src or (r and int(r.group(1)) <= int(src[1:]) <= int(r.group(2))):
                break
    return hits


def test_scan_finds_a_dropped_mask():
    asm = "\n".join([
        "_Zkern:",
        "\tv_and_b32_e32 v8, 0xffffff, v11",
        "\tv_mad_u64_u32 v[62:63], s[2:3], v11, 24, s[36:37]",
        "\tv_mad_u64_u32 v[60:61], s[2:3], v8, 24, s[36:37]",
    ])
    assert len(dropped_masks(asm)) == 1
    assert dropped_masks(asm.replace("v11, 24", "v8, 24")) == []


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
def test_no_dropped_index_mask_in_compute_kernels():
    src = os.path.join(ROOT, "paper_1710_00882_amd", "csrc", "compute.hip")
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "compute.s")
        cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I", os.path.join(ROOT, "include"), "-I", os.path.dirname(src),
               "--cuda-device-only", "-S", src, "-o", out]
        subprocess.run(cmd, check=True, capture_output=True)
        asm = open(out).read()
    assert "k_tersoff" in asm
    assert dropped_masks(asm) == []
