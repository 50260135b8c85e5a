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


@pytest.hookimpl(trylast=True)  # after -m has deselected items
def pytest_collection_modifyitems(config, items):
    """When GPU tests will run, initialise torch's HIP runtime before anything
    loads libgpe.so: torch ships its own copy of the runtime under the same
    soname, and the library must bind to the one torch has loaded (a GPU test
    that uses torch tensors next to the library needs that order)."""
    if any(item.get_closest_marker("gpu") for item in items):
        import torch

        if torch.cuda.is_available():
            torch.cuda.init()
