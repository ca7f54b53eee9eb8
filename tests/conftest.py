import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu on a machine that has one)")
    config.addinivalue_line("markers", "slow: longer CPU-side check")


@pytest.fixture(scope="session", autouse=True)
def _build_oracle_once():
    from oracle.oracle import build_oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "libmithra_oracle.so")):
        build_oracle()
    yield
