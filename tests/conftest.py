import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def load_primes():
    path = os.path.join(ROOT, "tests", "golden", "primes_1024.txt")
    with open(path) as f:
        return [int(l, 16) for l in f if l.strip() and not l.startswith("#")]


@pytest.fixture(scope="session")
def primes_1024():
    return load_primes()
