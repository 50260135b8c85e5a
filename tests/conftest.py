import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long CPU-only check (still part of the CPU suite)")


def load_golden(name):
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", name)
    return np.loadtxt(path, comments="#")


@pytest.fixture(scope="session")
def golden():
    return load_golden
