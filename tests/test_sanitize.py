"""Sanitizer builds of host code (CPU only; no GPU code is built with a
sanitizer).

* The oracle (oracle/oracle.c) with AddressSanitizer and
  UndefinedBehaviorSanitizer, driven by tests/sanitize/oracle_driver.c over
  every entry point, with work arrays of exactly the documented sizes.
* libtri's API layer (the host side of the C ABI: validation, contexts,
  workspace, plans, schedules, graphs) built for the CPU with g++ against a
  stand-in HIP runtime whose kernel launchers only count launches
  (tests/sanitize/hip_stub, api_stubs.cpp), with the same sanitizers, driven
  by tests/sanitize/api_driver.cpp: every refusal launches and allocates
  nothing and leaves the data as it was, solves never allocate or wait,
  every allocation is released.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(exe, tmp_path):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env, cwd=tmp_path)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", *SAN, "-Wall", "-Wno-unknown-pragmas",
                           os.path.join(ROOT, "oracle", "oracle.c"),
                           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe, "-lm"])
    r = _run(exe, tmp_path)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_api_layer_under_asan_ubsan(tmp_path):
    # the API source is copied to a .cpp name: a plain C++ translation unit
    # built by the host compiler (it holds no device code)
    src = tmp_path / "tri_api.cpp"
    shutil.copy(os.path.join(ROOT, "paper_1812_01178_amd", "csrc", "tri_api.hip"), src)
    san = os.path.join(ROOT, "tests", "sanitize")
    exe = str(tmp_path / "api_asan")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", *SAN, "-Wall", "-Wno-unused-function",
                           "-I" + os.path.join(san, "hip_stub"), "-I" + os.path.join(ROOT, "include"),
                           "-I" + os.path.join(ROOT, "paper_1812_01178_amd", "csrc"), str(src),
                           os.path.join(san, "api_stubs.cpp"), os.path.join(san, "api_driver.cpp"), "-o", exe,
                           "-ldl"])
    r = _run(exe, tmp_path)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
