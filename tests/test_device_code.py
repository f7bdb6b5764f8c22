"""The built library's device code holds no packed FP32 VALU instructions
(v_pk_add_f32, v_pk_mul_f32, v_pk_fma_f32): every HIP source is compiled with
the packed-FP32 target feature switched off and the kernels are written for
scalar FP32/FP64 issue.  The pair loops that raise a wave's issue priority
around each exponential lower it again: in every kernel the raises and the
lowerings come in equal numbers.  Reads only the library built in this tree
(its .hip_fatbin section, one offload bundle per source) and disassembles the
gfx950 code objects with the ROCm LLVM tools; no GPU is needed."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1505_01998_amd", "libkde_bw.so")
LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _tools():
    need = [shutil.which("objcopy"), os.path.join(LLVM, "clang-offload-bundler"), os.path.join(LLVM, "llvm-objdump")]
    return all(p and os.path.exists(p) for p in need)


def _disassemble(tmp_path):
    """The disassembly of every gfx950 code object in the library."""
    fat = tmp_path / "fatbin.bin"
    subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", LIB, str(fat)], check=True)
    data = fat.read_bytes()
    starts = [m.start() for m in re.finditer(re.escape(MAGIC), data)] + [len(data)]
    assert len(starts) > 1
    out = []
    for k in range(len(starts) - 1):
        part = tmp_path / f"b{k}.bin"
        part.write_bytes(data[starts[k]:starts[k + 1]])
        co = tmp_path / f"b{k}.co"
        subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o", f"--input={part}",
                        "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"], check=True)
        out.append(subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", str(co)], check=True,
                                  capture_output=True, text=True).stdout)
    return out


needs_tools = pytest.mark.skipif(not os.path.exists(LIB) or not _tools(), reason="library or ROCm LLVM tools missing")


@needs_tools
def test_no_packed_fp32_instructions(tmp_path):
    kernels, packed = 0, []
    for dis in _disassemble(tmp_path):
        kernels += len(re.findall(r"^[0-9a-f]+ <", dis, flags=re.M))
        packed += re.findall(r"\bv_pk_(?:add|mul|fma)_f32\b", dis)
    assert kernels > 20
    assert not packed, f"{len(packed)} packed FP32 instructions in device code"


@needs_tools
def test_issue_priority_raised_and_lowered_in_pairs(tmp_path):
    found = {}
    for dis in _disassemble(tmp_path):
        for m in re.finditer(r"^[0-9a-f]+ <([^>]+)>:\n(.*?)(?=^[0-9a-f]+ <|\Z)", dis, flags=re.M | re.S):
            name, body = m.group(1), m.group(2)
            up = len(re.findall(r"\bs_setprio\s+(?:0x)?0*1\b", body))
            down = len(re.findall(r"\bs_setprio\s+(?:0x)?0+\b", body))
            if up or down:
                found[name] = (up, down)
    assert found, "no kernel raises its issue priority"
    for name, (up, down) in found.items():
        assert up == down and up > 0, (name, up, down)
    assert any("k_lscv_units_f32_queue" in n for n in found)
    assert any("k_psi_units_f32" in n for n in found)
