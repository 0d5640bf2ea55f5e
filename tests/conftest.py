import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_collection_finish(session):
    """Forks the oracle pool and queues the oracle jobs of the selected GPU tests, in run order.

    Collection initialises no GPU (test modules import torch inside fixtures only), so the fork
    happens before any device call.  A module lists its jobs in ORACLE_JOBS: test name -> a
    function that submits them (tests/oracle_pool.py)."""
    items = [it for it in session.items if it.get_closest_marker("gpu")]
    if not items or session.config.option.collectonly:
        return
    from tests import oracle_pool
    oracle_pool.start()
    done = set()
    for it in items:
        jobs = getattr(it.module, "ORACLE_JOBS", {})
        name = getattr(it, "originalname", it.name)
        key = (it.module.__name__, name)
        if name in jobs and key not in done:
            done.add(key)
            jobs[name]()


def pytest_sessionfinish(session, exitstatus):
    mod = sys.modules.get("tests.oracle_pool")
    if mod is not None:
        mod.stop()


def load_primes():
    path = os.path.join(ROOT, "tests", "golden", "primes_1024.txt")
    with open(path) as f:
        return [int(l, 16) for l in f if l.strip() and not l.startswith("#")]


@pytest.fixture(scope="session")
def primes_1024():
    return load_primes()
