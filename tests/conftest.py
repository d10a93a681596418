import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_keys_c1():
    import oracle
    import workloads as W
    return oracle.keygen(W.C1, W.KEY_SEED["C1"])


@pytest.fixture(scope="session")
def oracle_keys_c1_exact():
    import oracle
    import workloads as W
    return oracle.keygen(W.exact(W.C1), W.KEY_SEED["C1"])


@pytest.fixture(scope="session")
def oracle_keys_c2():
    import oracle
    import workloads as W
    return oracle.keygen(W.C2, W.KEY_SEED["C2"])
