import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU or GPU case")


@pytest.fixture(scope="session", autouse=True)
def _native_test_libs():
    """The generator and the oracle are small gcc builds; build them once if absent."""
    import gen
    import oracle
    gen.build(force=False)
    oracle.build(force=False)
