import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# the planted-mistake test (tests/test_oracle_mutants.py) runs the pins
# against an altered copy of the oracle package placed first on the path
if os.environ.get("ORACLE_PKG_OVERRIDE"):
    sys.path.insert(0, os.environ["ORACLE_PKG_OVERRIDE"])


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build()
    return oracle
