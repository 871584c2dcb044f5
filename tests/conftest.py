import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU test")


_CACHE = {}


def cached_problem(name, **kw):
    """Seeded problems are deterministic; build each one once per session."""
    from workloads import make_problem
    key = (name, tuple(sorted(kw.items())))
    if key not in _CACHE:
        _CACHE[key] = make_problem(name, **kw)
    return _CACHE[key]


@pytest.fixture(scope="session")
def cube8x16():
    return cached_problem("cube8x16")
