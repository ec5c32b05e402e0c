"""Build libsbmm.so (HIP, gfx950) in-tree.

    python -m paper_2105_04940_amd.build        # or build() from Python

Every HIP source under csrc/ is compiled for gfx950 into one shared library
next to this file. Packed-FP32 instructions are disabled for device code.
"""
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_NAME = "libsbmm.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose=False, jobs=None):
    """Compile every source to an object in parallel, then link."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = [
        f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
        "-I", os.path.join(ROOT, "include"),
        "-I", os.path.join(HERE, "csrc"),
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-result",
    ]
    cc = hipcc()
    procs = []
    objs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [cc, *common, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(text)
        elif verbose and text.strip():
            sys.stderr.write(text)
    if failed:
        raise RuntimeError("HIP compile failed: " + ", ".join(os.path.basename(f) for f in failed))
    tmp = LIB_PATH + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


SAN_LIB_PATH = os.path.join(HERE, "libsbmm_san.so")


def build_sanitized(verbose=False):
    """The same library with AddressSanitizer and UndefinedBehaviorSanitizer
    on the host code only (argument validation, workspace sizing, the arena,
    status handling); device code is built as usual. For CPU tests of the
    host paths: load it with the sanitizer runtime preloaded (see
    tests/test_host_sanitized.py)."""
    objdir = os.path.join(HERE, "_build_san")
    os.makedirs(objdir, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    common = [
        f"--offload-arch={ARCH}", "-O1", "-g", "-fPIC", "-std=c++17",
        "-I", os.path.join(ROOT, "include"),
        "-I", os.path.join(HERE, "csrc"),
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-result", *san,
    ]
    cc = hipcc()
    procs, objs = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [cc, *common, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(out.decode(errors="replace"))
    if failed:
        raise RuntimeError("sanitized HIP compile failed: " + ", ".join(os.path.basename(f) for f in failed))
    tmp = SAN_LIB_PATH + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SAN_LIB_PATH)
    return SAN_LIB_PATH


WORKLOAD_SRC = os.path.join(ROOT, "workloads", "gen.hip")
WORKLOAD_LIB = os.path.join(ROOT, "workloads", "libsbmm_workload.so")


def build_workload(verbose=False):
    """The device-side input generator (workloads/gen.hip), a library of its
    own: it generates test and benchmark inputs and is not part of libsbmm."""
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           WORKLOAD_SRC, "-o", WORKLOAD_LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(WORKLOAD_LIB + ".tmp", WORKLOAD_LIB)
    return WORKLOAD_LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    print(build_workload(verbose="-v" in sys.argv))
