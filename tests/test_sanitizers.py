"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): the
library's plan arithmetic (s2w_host.cpp, driven by csrc/host_check.cpp) and the oracle's C
core (oracle/wigner_oracle.c, driven by oracle/oracle_check.c), built with g++/gcc and run;
any sanitizer report or violated invariant fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, exe, tmp_path):
    if shutil.which(cmd[0]) is None:
        pytest.skip(f"{cmd[0]} not available")
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_host_plan_code_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2402_01282_amd", "csrc")
    exe = str(tmp_path / "host_check")
    out = _run(["g++", "-std=c++17", *SAN, "-I", csrc, os.path.join(csrc, "host_check.cpp"),
                os.path.join(csrc, "s2w_host.cpp"), "-o", exe, "-lpthread"], exe, tmp_path)
    assert "host_check ok" in out


def test_oracle_core_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    out = _run(["gcc", "-std=c11", *SAN, os.path.join(ROOT, "oracle", "oracle_check.c"),
                os.path.join(ROOT, "oracle", "wigner_oracle.c"), "-o", exe, "-lm"], exe, tmp_path)
    assert "oracle_check ok" in out
