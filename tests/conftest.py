import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the GPU)")
    config.addinivalue_line("markers", "slow: long-running (full-size workloads)")


@pytest.fixture(scope="session")
def orc():
    """The oracle; TPX_ORACLE_LIB points it at another build of the same
    source (the mutation test uses this to run the pins on planted bugs)."""
    import oracle
    path = os.environ.get("TPX_ORACLE_LIB")
    return oracle.Oracle(path) if path else oracle.get()
