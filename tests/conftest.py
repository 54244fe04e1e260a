import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


# Primes used across the tests: the largest prime below 2^b for b in
# {3 (=7), 20, 23, 25, 26, 31, 36, 40, 50, 52}, plus p = 5.
PRIMES = [5, 7, 1048573, 8388593, 33554393, 67108859, 2147483647, 68719476731,
          1099511627689, 1125899906842597, 4503599627370449]


@pytest.fixture(scope="session")
def primes():
    return list(PRIMES)
