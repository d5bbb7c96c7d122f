import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long CPU-side oracle work")


@pytest.fixture(scope="session")
def s32k():
    """The paper's parameters (N = 32768, 17 + 1 primes, t = 65537) with the
    keys of seed 0, shared by the full-size GPU test modules."""
    from tests.gpu_common import Setup
    return Setup(15)


@pytest.fixture(scope="session")
def s32k_a2():
    """The paper's size with key switching by digits of two data primes (16
    data primes, two special primes), keys of seed 0."""
    from tests.gpu_common import Setup
    return Setup(15, alpha=2)


@pytest.fixture(scope="session")
def s32k_a3():
    """The paper's size with key switching by digits of three data primes (15
    data primes, three special primes), keys of seed 0."""
    from tests.gpu_common import Setup
    return Setup(15, alpha=3)
