"""Memory and undefined-behaviour checks on the CPU: the oracle's C stepper
and the library's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; no device code is sanitized),
run on exact-size allocations.  The drivers are in tests/sanitize/."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2106_11476_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def test_oracle_stepper_is_clean_under_asan_and_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_asan")
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           "-fno-sanitize-recover=all", os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"])
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "108 of 108 clean" in r.stdout


def test_library_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    from paper_2106_11476_amd import build
    exe = str(tmp_path / "abi_asan")
    # each sanitizer flag is passed to the host compilation only
    san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer",
                 "-fno-sanitize-recover=all"):
        san += ["-Xarch_host", flag]
    cmd = [build.hipcc(), "-std=c++17", "-O1", "-g"] + san + [
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        os.path.join(CSRC, "fw2.cpp"), os.path.join(CSRC, "setup.cpp"),
        os.path.join(SAN, "launch_stubs.cpp"), os.path.join(SAN, "abi_driver.cpp"), "-o", exe]
    subprocess.check_call(cmd)
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failed" in r.stdout
