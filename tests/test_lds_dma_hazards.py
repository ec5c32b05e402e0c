"""Wait states of the inline-asm LDS-DMA loads (host only: compiles, runs nothing).

The matrix-core kernels load their operand tiles with an inline-asm
``buffer_load_dwordx4 ... offen lds``. The compiler inserts the wait states a
GFX9-family load needs after its operands are written only for instructions
it can see, not inside inline asm, so the asm carries them: one for the m0
write just before it, and five more wherever an operand SGPR may have just
been written by a vector instruction (a readfirstlane of a value held in
vector registers). A load that reads such an SGPR too soon takes a stale
resource, offset or LDS base. This test compiles the kernel sources to
gfx950 assembly and checks, for every such load, that its own s_nop is there
and that no vector instruction writes an SGPR it reads within the five wait
states before it.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2105_04940_amd", "csrc")
SOURCES = ["hgemm.hip", "gemm.hip"]   # the kernels that load through the inline asm
LOAD = re.compile(r"buffer_load_dwordx4 v\d+, (s\[\d+:\d+\]), (s\d+) offen lds")


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def _sgprs(op):
    m = re.fullmatch(r"s\[(\d+):(\d+)\]", op)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.fullmatch(r"s(\d+)", op)
    return {int(m.group(1))} if m else set()


def _valu_sgpr_dest(ins):
    """SGPRs a vector instruction writes (readfirstlane, readlane, compares
    into an SGPR pair), else the empty set."""
    if not ins.startswith("v_"):
        return set()
    parts = ins.split(None, 1)
    if len(parts) < 2:
        return set()
    first = parts[1].split(",")[0].strip()
    return _sgprs(first)


def _instructions(asm):
    """(instruction, inside an inline-asm block) in order; loads that the
    compiler emits itself (the load-to-LDS builtin) get its own hazard
    handling and are not checked."""
    out = []
    in_asm = False
    for line in asm.splitlines():
        t = line.strip()
        if t.startswith(";;#ASMSTART"):
            in_asm = True
            continue
        if t.startswith(";;#ASMEND"):
            in_asm = False
            continue
        if not t or t.startswith((";", ".")) or t.endswith(":"):
            continue
        out.append((t.split(";")[0].strip(), in_asm))
    return out


@pytest.fixture(scope="module")
def assembly(tmp_path_factory):
    """gfx950 assembly of each source, compiled in parallel."""
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    tmp = tmp_path_factory.mktemp("asm")
    procs = {}
    for src in SOURCES:
        out = tmp / (src + ".s")
        cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
               "--cuda-device-only", "-S", "-o", str(out), os.path.join(CSRC, src)]
        procs[src] = (subprocess.Popen(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE), out)
    texts = {}
    for src, (proc, out) in procs.items():
        _, err = proc.communicate()
        assert proc.returncode == 0, err.decode()[-2000:]
        texts[src] = out.read_text()
    return texts


@pytest.mark.parametrize("src", SOURCES)
def test_lds_dma_loads_have_their_wait_states(src, assembly):
    tagged = _instructions(assembly[src])
    ins = [t for t, _ in tagged]
    loads = 0
    for i, (t, in_asm) in enumerate(tagged):
        m = LOAD.fullmatch(t)
        if not m or not in_asm:
            continue
        loads += 1
        used = _sgprs(m.group(1)) | _sgprs(m.group(2))
        # the asm's own s_nop comes right before the load
        assert i > 0 and ins[i - 1].startswith("s_nop"), f"{src}: LDS-DMA load without its s_nop: {t}"
        waits = int(ins[i - 1].split()[1]) + 1
        j = i - 2
        while waits < 5 and j >= 0:
            prev = ins[j]
            hit = _valu_sgpr_dest(prev) & used
            assert not hit, f"{src}: '{prev}' writes s{sorted(hit)} {waits} wait states before '{t}'"
            m2 = re.fullmatch(r"s_nop (\d+)", prev)
            waits += int(m2.group(1)) + 1 if m2 else 1
            j -= 1
    assert loads > 0, f"{src}: no LDS-DMA loads found"
