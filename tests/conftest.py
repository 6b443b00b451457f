import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running oracle checks")


_CACHE = {}


def cached(key, fn):
    """Process-wide cache for oracle systems / ground states (tests only)."""
    if key not in _CACHE:
        _CACHE[key] = fn()
    return _CACHE[key]


@pytest.fixture(scope="session")
def oracle_case():
    """oracle_case(name) -> (System, GroundState), cached per session."""
    from oracle.groundstate import ground_state
    from oracle.system import System
    from workloads import config

    def get(name):
        return cached(("gs", name), lambda: (lambda s: (s, ground_state(s)))(
            System(config(name))))
    return get
