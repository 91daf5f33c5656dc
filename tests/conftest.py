import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def lib():
    """The built rendering library (ctypes), or skip when it has not been built."""
    from paper_1205_0282_amd import binding
    try:
        return binding.load_library()
    except binding.LibraryMissing as e:  # pragma: no cover - depends on build state
        pytest.skip(str(e))
