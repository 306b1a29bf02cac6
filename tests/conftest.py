import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(autouse=True)
def _no_planted_fault():
    """Every test starts and ends with the oracle's planted-fault hook off."""
    import oracle
    oracle.set_fault(0)
    yield
    oracle.set_fault(0)
