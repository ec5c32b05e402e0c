"""The host code of the C ABI (argument validation, size queries, workspace
sizing, status strings) under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/test_abi.py and tests/test_host_sizes.py run in a child process against
libsbmm_san.so (the library with both sanitizers on its host code, built by
paper_2105_04940_amd.build.build_sanitized and __graft_entry__.build), with the
sanitizer runtime preloaded and any report fatal. CPU only: no device call is
made."""
import glob
import os
import subprocess
import sys

import pytest

import paper_2105_04940_amd.build as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    for pat in ("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so",
                "/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"):
        hits = sorted(glob.glob(pat))
        if hits:
            return hits[-1]
    return None


def test_host_paths_clean_under_asan_ubsan(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no clang sanitizer runtime in this image")
    if not os.path.exists(b.SAN_LIB_PATH):
        pytest.skip("libsbmm_san.so not built (paper_2105_04940_amd.build.build_sanitized)")
    log = str(tmp_path / "san")
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, SBMM_LIB=b.SAN_LIB_PATH,
               ASAN_OPTIONS=f"detect_leaks=0:abort_on_error=1:log_path={log}",
               UBSAN_OPTIONS=f"print_stacktrace=1:halt_on_error=1:log_path={log}")
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_abi.py"), os.path.join(ROOT, "tests", "test_host_sizes.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    reports = "".join(open(f).read() for f in glob.glob(log + "*"))
    assert r.returncode == 0 and not reports, (r.stdout[-2000:], r.stderr[-2000:], reports[-4000:])
    assert " passed" in r.stdout
