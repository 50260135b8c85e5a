"""Host code under the address and undefined-behaviour sanitizers (CPU only):
the oracle, driven through every entry point on small grids, and the request
server's scheduling policy (admission order and tiers, chunk sizes).  Each
program is built with g++ and must run to its OK line; a sanitizer report
stops it with a non-zero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def build_and_run(tmp_path, name, sources, includes, ok_line):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror"] + SAN + \
          ["-I" + i for i in includes] + sources + ["-o", exe, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert ok_line in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_oracle_under_sanitizers(tmp_path):
    build_and_run(tmp_path, "oracle_sanitize",
                  [os.path.join(ROOT, "tests", "c", "oracle_sanitize.cpp"),
                   os.path.join(ROOT, "oracle", "oracle.cpp")],
                  [os.path.join(ROOT, "oracle")], "oracle sanitize OK")


def test_scheduling_policy_under_sanitizers(tmp_path):
    build_and_run(tmp_path, "sched_policy_check",
                  [os.path.join(ROOT, "tests", "c", "sched_policy_check.cpp")],
                  [os.path.join(ROOT, "paper_2301_08275_amd", "csrc")], "sched policy OK")
