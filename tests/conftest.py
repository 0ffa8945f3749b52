import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


def read_golden(name):
    """Lines of a golden fixture with comments and blank lines removed."""
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.strip() for ln in fh if ln.strip() and not ln.startswith("#")]


@pytest.fixture
def golden():
    return read_golden
