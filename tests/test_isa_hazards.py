"""The decoder kernels' gfx950 code reads no MFMA result too early (CPU only).

A VALU instruction that reads a VGPR written by an MFMA needs a number of
independent instructions (wait states) after it: about the MFMA's pass count
plus four on CDNA3/4 (8-pass 32x32x16 bf16: 12; 16-pass 32x32x2 f32: 20).
The compiler is meant to insert them, but it was seen to leave an integer
med3 of the accumulator bits four instructions after the last MFMA of a
tile, which read stale accumulators.  Every GEMM therefore ends with explicit
wait states; this test compiles the kernels to assembly and checks, within
each basic block, every VALU read of a 32x32 MFMA result.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1911_13225_amd", "csrc", "mlp_kernels.hip")


def _vregs(op):
    m = re.match(r"v\[(\d+):(\d+)\]", op)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", op)
    return {int(m.group(1))} if m else set()


def scan(asm):
    """(kernel, instruction, wait states) of every VALU read of a 32x32 MFMA
    destination with fewer wait states than required since the MFMA; s_nop N
    counts N + 1, every other instruction 1; a label ends the block."""
    bad = []
    for km in re.finditer(r"^(\S+):[^\n]*\n", asm, re.M):
        name = km.group(1)
        if name.startswith("."):
            continue
        end = asm.find(".Lfunc_end", km.end())
        if end < 0:
            continue
        pend = None          # [destination registers, wait states so far, required]
        for line in asm[km.end():end].split("\n"):
            t = line.split(";")[0].strip()
            if not t:
                continue
            if t.startswith("."):
                if re.match(r"^\.LBB\w*:", t):
                    pend = None
                continue
            ins = t.split()[0]
            ops = [o.strip() for o in t[len(ins):].split(",")]
            if ins.startswith("v_mfma_f32_32x32"):
                pend = [_vregs(ops[0]), 0, 20 if ins.endswith("f32_32x32x2f32") or ins.endswith("x2_f32") else 12]
                continue
            if pend is None:
                continue
            if ins == "s_nop":
                pend[1] += int(ops[0], 0) + 1
                continue
            if ins.startswith("v_"):
                src = set()
                for o in ops[1:]:
                    src |= _vregs(o)
                if src & pend[0] and pend[1] < pend[2]:
                    bad.append((name, t, pend[1]))
                    pend = None
                    continue
            pend[1] += 1
    return bad


def test_scan_flags_an_early_read_and_accepts_a_drained_one():
    head = "k:\n\tv_mfma_f32_32x32x16_bf16 v[2:17], v[18:21], v[22:25], v[2:17]\n"
    early = head + "\tv_lshrrev_b32_e32 v19, 5, v43\n" * 4 + "\tv_med3_i32 v19, v2, 0, 1\n.Lfunc_end0:\n"
    drained = head + "\ts_nop 7\n\ts_nop 7\n\tv_med3_i32 v19, v2, 0, 1\n.Lfunc_end0:\n"
    other = head + "\tv_med3_i32 v19, v40, 0, 1\n.Lfunc_end0:\n"
    f32 = ("k:\n\tv_mfma_f32_32x32x2f32 v[2:17], v18, v19, v[2:17]\n\ts_nop 7\n\ts_nop 7\n"
           "\tv_max_f32_e32 v3, v3, v3\n.Lfunc_end0:\n")
    assert [b[2] for b in scan(early)] == [4]
    assert scan(drained) == [] and scan(other) == []
    assert [b[2] for b in scan(f32)] == [16]


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_decoder_kernels_read_no_mfma_result_early(tmp_path):
    import importlib.util
    spec = importlib.util.spec_from_file_location("dist_build", os.path.join(ROOT, "paper_1911_13225_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    flags = [f for f in b.FLAGS if f != "-fPIC"]
    out = str(tmp_path / "mlp.s")
    r = subprocess.run([b.HIPCC, *flags, "--cuda-device-only", "-S", SRC, "-o", out], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    asm = open(out).read()
    assert asm.count("v_mfma_f32_32x32x16_bf16") > 100
    bad = scan(asm)
    assert not bad, bad[:5]
