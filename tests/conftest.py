import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: full-size workloads (minutes on the CPU)")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import oracle as O
    O.build(force=False)
    return O


_EVENTS = {}


def cached_event(name, factory):
    if name not in _EVENTS:
        _EVENTS[name] = factory()
    return _EVENTS[name]
