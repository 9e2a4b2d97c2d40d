import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import oracle as orc
    if not os.path.exists(orc._LIB_PATH) or os.path.getmtime(orc._LIB_PATH) < os.path.getmtime(orc._SRC):
        orc.build(force=True)
    yield
