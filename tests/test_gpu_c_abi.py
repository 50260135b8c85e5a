"""The C ABI called from a plain C program (no Python, no torch): a 2D
Table 1 ground state and 100 real-time steps."""
import os
import subprocess
import sys

import pytest

from paper_2301_08275_amd import gpe

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_program_through_the_abi(tmp_path):
    exe = str(tmp_path / "abi_demo")
    libdir = os.path.dirname(gpe.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-O2", os.path.join(ROOT, "tests", "c", "abi_demo.c"),
           "-I", os.path.join(ROOT, "include"), "-L", libdir, "-lgpe",
           "-Wl,-rpath," + libdir, "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    print("running", exe, flush=True)
    sys.stdout.flush()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.stdout, r.stderr)
    st, steps, energy, mu, norm = r.stdout.split()
    assert int(st) == 0 and int(steps) > 0
    # Table 1, 2D, g = 12.5484: mu = 2.25609 (this scheme at dt = 1e-3: 2.25610)
    assert abs(float(mu) / 2.25609 - 1) < 1e-4
    assert abs(float(norm) - 1) < 1e-12
