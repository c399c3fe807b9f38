import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    """The CPU reference (built on demand)."""
    import oracle
    oracle.load()
    return oracle


@pytest.fixture(scope="session")
def F():
    from paper_1410_1942_amd import fields
    return fields
