import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import build as oracle_build
    import oracle
    src_time = max(os.path.getmtime(os.path.join(oracle.HERE, f))
                   for f in ("oracle.cpp", "brute.cpp", "graph_internal.h", "timest_oracle.h"))
    if not os.path.exists(oracle.LIB_PATH) or os.path.getmtime(oracle.LIB_PATH) < src_time:
        oracle_build.build()
    yield
