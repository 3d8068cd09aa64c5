import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def large_oracle_map():
    """Oracle counts and binary32 map of the large workload (32768^2 rays, 2048^2)."""
    import workloads as W
    from tests.helpers import note, oracle_map
    c = W.config("large")
    note("oracle map large (C mirror, 16 threads)")
    return oracle_map(c["s"], c["q"], c["rays"], c["window"], c["rho"])


@pytest.fixture(scope="session")
def tiny_oracle_map():
    import workloads as W
    from tests.helpers import oracle_map
    c = W.config("tiny")
    return oracle_map(c["s"], c["q"], c["rays"], c["window"], c["rho"])
