import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device); run with -m gpu")
    config.addinivalue_line("markers", "slow: full-size inputs (minutes on one host core)")


@pytest.fixture(scope="session", autouse=True)
def _built_helpers():
    """Compile the CPU helpers (generators, oracle) if they are not built."""
    import graphgen
    import oracle
    graphgen.build(force=False)
    oracle.build(force=False)
    yield
