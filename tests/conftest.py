import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


def pytest_runtest_setup(item):
    # name each GPU test before it runs, unbuffered, so that a run that dies
    # in a device call still shows which test it was in
    if item.get_closest_marker("gpu") is not None:
        sys.__stderr__.write(f"[start] {item.nodeid}\n")
        sys.__stderr__.flush()
