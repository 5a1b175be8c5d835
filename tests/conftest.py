import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# The mutation tests point this at a directory holding a deliberately broken copy of the
# oracle package, which must shadow the real one.
if os.environ.get("TREEPM_ORACLE_PKG"):
    sys.path.insert(0, os.environ["TREEPM_ORACLE_PKG"])


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle
