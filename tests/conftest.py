import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libcox.so")
    config.addinivalue_line("markers", "slow: full-size case (minutes on the CPU)")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle

    oracle.lib()
    oracle.set_threads(min(8, os.cpu_count() or 1))
    return oracle
