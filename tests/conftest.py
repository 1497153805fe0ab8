import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def cfg1():
    from paper_2608_17844_amd import workloads as W
    return W.cpu_size_5x5()


@pytest.fixture(scope="session")
def cfg1_dense(cfg1):
    from oracle import mom
    return mom.fill_dense(cfg1.lattice, cfg1.dipole, 1.0)


@pytest.fixture(scope="session")
def cfg1_oracle(cfg1):
    from oracle import mom
    return mom.solve_array(cfg1.lattice, cfg1.dipole, 1.0, cfg1.theta, cfg1.phi, keep_Z=True)
