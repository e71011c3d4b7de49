import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def lib():
    """The built C-ABI library (skips when it has not been built)."""
    from paper_2007_00789_amd import spand
    try:
        return spand.load()
    except OSError as e:  # not built here
        pytest.skip(f"libspand not built: {e}")
