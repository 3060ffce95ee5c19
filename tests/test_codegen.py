"""Checks of this library's own compiled gfx950 code (CPU only): the device code object is
unbundled from the built kernels object and disassembled with the ROCm LLVM tools.

The binary32 P_z step loop (the bench workload's kernel) must start on a 32-byte boundary:
measured on the MI355X, the same loop at offset 44 of a 64-byte line ran 7 % slower than at
offsets 0 and 32 (same instructions, same registers per lane).  And its VALU instruction
count must equal the per-step count the roofline charges, class by class where the classes
cost differently (transcendentals, 32x32->64 multiplies, conversions, binary64 work), so
that the bench line's count is the compiled loop's."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_1703_08977_amd import roofline
from paper_1703_08977_amd import workloads as W

from hefk_testutil import CSRC

LLVM = "/opt/rocm/lib/llvm/bin"
OBJ = os.path.join(CSRC, "_build", "hefk_kernels.o")
MIXED_PZ = "_ZN4hefk16propagate_kernelIfLi3ELi1ELb0EEEvNS_5KArgsE"  # <float, P_z, Gaussian contract 2, no variants>


def _tool(name):
    p = os.path.join(LLVM, name)
    return p if os.path.exists(p) else shutil.which(name)


@pytest.fixture(scope="module")
def disassembly():
    tools = [_tool(t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-objdump")]
    if not os.path.exists(OBJ) or not all(tools):
        pytest.skip("kernels object or ROCm LLVM tools not present (build the library first)")
    objcopy, bundler, objdump = tools
    d = tempfile.mkdtemp(prefix="hefk_codegen_")
    fat, co = os.path.join(d, "fatbin"), os.path.join(d, "gfx950.co")
    subprocess.check_call([objcopy, "--dump-section", ".hip_fatbin=" + fat, OBJ])
    subprocess.check_call([bundler, "--type=o", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", "--input=" + fat,
                           "--output=" + co, "--unbundle"])

    def dis(symbol):
        return subprocess.run([objdump, "-d", "--no-show-raw-insn", "--disassemble-symbols=" + symbol, co],
                              capture_output=True, text=True, check=True).stdout
    return dis


def _innermost_loop(text, ops=False):
    """(branch target address, VALU instructions) of the smallest backward-branch loop holding
    more than 50 VALU instructions (with ops: the loop's VALU mnemonics instead of their count)."""
    insts = []
    for line in text.split("\n"):
        m = re.match(r"\s+(\w+)\s*(.*?)//\s*([0-9A-F]+):", line)
        if m:
            insts.append((int(m.group(3), 16), m.group(1), line))
    start = insts[0][0]
    best = None
    for addr, op, line in insts:
        if op.startswith("s_cbranch") or op == "s_branch":
            m = re.search(r"\+0x([0-9a-f]+)>", line)
            if m and start + int(m.group(1), 16) < addr:
                tgt = start + int(m.group(1), 16)
                body = [o for a, o, _ in insts if tgt <= a <= addr and o.startswith("v_")]
                if len(body) > 50 and (best is None or len(body) < best[1]):
                    best = (tgt, len(body), body)
    return (best[0], best[2]) if ops else best[:2]


def test_bench_step_loop_is_32_byte_aligned(disassembly):
    tgt, n = _innermost_loop(disassembly(MIXED_PZ))
    assert tgt % 32 == 0, "step loop at offset %d of a 64-byte line" % (tgt % 64)


def test_bench_step_loop_instruction_count_is_the_roofline_count(disassembly):
    _, n = _innermost_loop(disassembly(MIXED_PZ))
    assert n == roofline.instructions_per_walker_step(W.get("he_2P_pz_16m")), n


def _classes(mnemonics):
    out = {"trans": 0, "mad": 0, "cvt": 0, "cvt64": 0, "f64": 0, "other": 0}
    for o in mnemonics:
        if re.match(r"v_(sqrt|rsq|rcp|log|exp|sin|cos)_f32", o):
            out["trans"] += 1
        elif o.startswith("v_mad_u64_u32"):
            out["mad"] += 1
        elif o.startswith("v_cvt") and "f64" in o:
            out["cvt64"] += 1
        elif o.startswith("v_cvt"):
            out["cvt"] += 1
        elif re.match(r"v_\w+_f64", o):
            out["f64"] += 1
        else:
            out["other"] += 1
    return out


def test_bench_step_loop_classes_are_the_roofline_classes(disassembly):
    _, body = _innermost_loop(disassembly(MIXED_PZ), ops=True)
    got = _classes(body)
    want = roofline.class_counts(W.get("he_2P_pz_16m"))
    for cls in ("trans", "mad", "cvt", "cvt64", "f64"):
        assert got[cls] == want.get(cls, 0), (cls, got, want)
    assert got["other"] == want.get("a32", 0) + want.get("sel", 0), (got, want)
