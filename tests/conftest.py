import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test (tens of seconds)")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def tiny_world():
    import synth.configs as C
    return C.make("tiny", noise=False)


@pytest.fixture(scope="session")
def tiny_eta(tiny_world, oracle_lib):
    return oracle_lib.observed_field_angles(tiny_world)
