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


def check(asm):
    """Problems of the inline-asm LDS-DMA loads in an assembly text (empty
    when every load has its wait states) and the number of such loads."""
    tagged = _instructions(asm)
    ins = [t for t, _ in tagged]
    problems, loads = [], 0
    for i, (t, in_asm) in enumerate(tagged):
        m = LOAD.fullmatch(t)
        if not m or not in_asm:
            continue
        loads += 1
        used = _sgprs(m.group(1)) | _sgprs(m.group(2))
        # the asm's own s_nop comes right before the load
        if i == 0 or not ins[i - 1].startswith("s_nop"):
            problems.append(f"load without its s_nop: {t}")
            continue
        waits = int(ins[i - 1].split()[1]) + 1
        j = i - 2
        while waits < 5 and j >= 0:
            prev = ins[j]
            hit = _valu_sgpr_dest(prev) & used
            if hit:
                problems.append(f"'{prev}' writes s{sorted(hit)} {waits} wait states before '{t}'")
            m2 = re.fullmatch(r"s_nop (\d+)", prev)
            waits += int(m2.group(1)) + 1 if m2 else 1
            j -= 1
    return problems, loads


@pytest.mark.parametrize("src", SOURCES)
def test_lds_dma_loads_have_their_wait_states(src, assembly):
    problems, loads = check(assembly[src])
    assert loads > 0, f"{src}: no LDS-DMA loads found"
    assert not problems, f"{src}: " + "; ".join(problems[:5])


def _asm_load(pre, nop=0):
    """A synthetic instruction sequence ending in one inline-asm load that
    reads s[8:11] and s4."""
    body = "\n".join(f"\t{x}" for x in pre)
    return (f"{body}\n\t;;#ASMSTART\n\ts_nop {nop}\n"
            "\tbuffer_load_dwordx4 v1, s[8:11], s4 offen lds\n\t;;#ASMEND\n")


def test_checker_flags_planted_hazards():
    # a readfirstlane into the resource right before the load
    assert check(_asm_load(["v_readfirstlane_b32 s10, v2", "s_mov_b32 m0, s3"]))[0]
    # into the soffset, three instructions before
    assert check(_asm_load(["v_readfirstlane_b32 s4, v2", "s_add_u32 s5, s5, 1", "s_mov_b32 m0, s3"]))[0]
    # a compare into an SGPR pair the resource uses
    assert check(_asm_load(["v_cmp_eq_u32_e64 s[8:9], v1, v2", "s_mov_b32 m0, s3"]))[0]
    # a load without its own s_nop
    assert check("\t;;#ASMSTART\n\tbuffer_load_dwordx4 v1, s[8:11], s4 offen lds\n\t;;#ASMEND\n")[0]


def test_checker_accepts_settled_operands():
    # the same writes, but five wait states before the load (the asm's own
    # s_nop 4), or far enough back, or to SGPRs the load does not read
    assert not check(_asm_load(["v_readfirstlane_b32 s10, v2", "s_mov_b32 m0, s3"], nop=4))[0]
    assert not check(_asm_load(["v_readfirstlane_b32 s10, v2"] + ["s_add_u32 s5, s5, 1"] * 4 + ["s_mov_b32 m0, s3"]))[0]
    assert not check(_asm_load(["v_readfirstlane_b32 s12, v2", "s_mov_b32 m0, s3"]))[0]
    # a load the compiler emits itself (no inline-asm markers) is its own business
    assert check("\tv_readfirstlane_b32 s10, v2\n\tbuffer_load_dwordx4 v1, s[8:11], s4 offen lds\n") == ([], 0)
