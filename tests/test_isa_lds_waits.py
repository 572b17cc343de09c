"""Static check of the matrix-core correlation kernels' gfx950 assembly.

Its LDS reads are inline asm (the compiler cannot count the direct
global->LDS DMA completions across the stage loop, so the waits are explicit).
This test compiles the kernel and verifies that no instruction reads or
overwrites a VGPR that an inline-asm ds_read_b128 is still filling, i.e. that
every consumer comes after an `s_waitcnt lgkmcnt(0)`."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1312_6182_amd", "csrc")


def _regs(tok):
    m = re.match(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def lds_read_hazards(body_lines):
    pending, bad = set(), []
    for line in body_lines:
        t = line.strip()
        if not t or t[0] in ";." or t.endswith(":"):
            continue
        op = t.split()[0]
        args = [a.strip() for a in t[len(op):].split(",")]
        if op == "s_waitcnt" and "lgkmcnt(0)" in t:
            pending.clear()
            continue
        if op == "ds_read_b128":
            pending |= _regs(args[0])
            continue
        if op.startswith(("v_", "global_", "ds_", "buffer_")):
            srcs = set()
            for a in args[1:]:
                if a:
                    srcs |= _regs(a.split()[0])
            if srcs & pending or (args and _regs(args[0]) & pending):
                bad.append(t)
    return bad


def test_checker_flags_a_consumer_before_the_wait():
    body = ["ds_read_b128 v[4:7], v1", "v_mfma_f32_16x16x4_f32 a[0:3], v4, v8, a[0:3]",
            "s_waitcnt lgkmcnt(0)"]
    assert lds_read_hazards(body)
    ok = ["ds_read_b128 v[4:7], v1", "s_waitcnt lgkmcnt(0)",
          "v_mfma_f32_16x16x4_f32 a[0:3], v4, v8, a[0:3]"]
    assert not lds_read_hazards(ok)


@pytest.mark.skipif(not (os.path.exists("/opt/rocm/bin/hipcc") or shutil.which("hipcc")),
                    reason="hipcc not installed")
@pytest.mark.parametrize("src,kernel,mfma,count", [
    ("k_corr_mfma.hip", "k_corr_mfma", "v_mfma_f32_16x16x4_f32", 4),
    ("k_corr_mfma.hip", "k_corr_wg", "v_mfma_f32_16x16x4_f32", 3),
    ("k_quant.hip", "k_corr_q", "v_mfma_f32_16x16x32_bf16", 6),
])
def test_mfma_kernel_waits_before_consuming_lds_reads(tmp_path, src, kernel, mfma, count):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    out = tmp_path / "k.s"
    cmd = [hipcc, "-x", "hip", "-S", "--cuda-device-only", "--offload-arch=gfx950", "-O3",
           "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), os.path.join(CSRC, src), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    asm = out.read_text()
    names = re.findall(r"^(_Z\S*" + kernel + r"\S*):", asm, re.M)
    assert len(names) >= count
    for name in names:
        i = asm.find(name + ":")
        j = asm.find(".Lfunc_end", i)
        body = asm[i:j].split("\n")
        assert any(mfma in l for l in body)
        assert any("global_load_lds_dwordx4" in l for l in body)
        assert lds_read_hazards(body) == [], name
