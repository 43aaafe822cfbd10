"""The host code of libmera.so (argument checks, the contraction planner, the measuring
pass that sizes workspaces, plan strings) under AddressSanitizer and UBSan.

The library is rebuilt with the host sanitizers (device code unchanged) into a temporary
directory, and the CPU tests of the C ABI run against it in a child process with the
sanitizer runtime preloaded; any report ends that process with an error.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    pats = ("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so",
            "/opt/rocm*/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    for pat in pats:
        hits = sorted(glob.glob(pat))
        if hits:
            return hits[-1]
    return None


@pytest.mark.slow
def test_abi_checks_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    runtime = _asan_runtime()
    if runtime is None:
        pytest.skip("no AddressSanitizer runtime in the ROCm toolchain")
    from paper_1906_12030_amd import build

    lib = build.build(sanitize=True, out_dir=str(tmp_path))
    env = dict(os.environ)
    env.update(
        LD_PRELOAD=runtime,
        MERA_LIBRARY=lib,
        ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
        UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
    )
    cmd = [sys.executable, "-m", "pytest", "-q", "-s", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_abi.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    log = r.stdout[-6000:] + r.stderr[-6000:]
    assert r.returncode == 0, log
    assert "passed" in r.stdout and "skipped" not in r.stdout, log
    assert "runtime error" not in log and "AddressSanitizer" not in log, log
