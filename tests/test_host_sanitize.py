"""The C ABI's host code under ASan and UBSan (CPU only).

tests/host_sanitize/bookkeeping_driver.cpp compiles the library's host code into a
program that drives problem definition, bookkeeping, the Schur-complement pair
structure and the workspace layout of every landmark-block form on random and
degenerate inputs; no GPU call is made.  tests/host_sanitize/lm_driver.cpp runs
the whole host side (creation, upload, autotuner, stages, LM loop) with the HIP
runtime replaced by a host stand-in and the kernel launchers by no-ops.  The
sanitizers apply to host code only.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_bookkeeping_under_sanitizers(tmp_path):
    exe = str(tmp_path / "bookkeeping_driver")
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host_sanitize", "bookkeeping_driver.cpp"),
           "-Wl,--unresolved-symbols=ignore-all", "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "cases ok" in run.stdout


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_lm_loop_under_sanitizers(tmp_path):
    exe = str(tmp_path / "lm_driver")
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host_sanitize", "lm_driver.cpp"),
           "-Wl,--unresolved-symbols=ignore-all", "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "cases ok" in run.stdout
