import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.num_threads()  # loads (and builds if missing) liboracle.so
    return oracle


@pytest.fixture(scope="session")
def synth():
    from paper_2206_08301_amd import synth as s
    return s
