import functools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def golden_path(name):
    return os.path.join(GOLDEN, name)


@functools.lru_cache(maxsize=None)
def oracle_bura(alpha, k, m=None, beta=1):
    """Session-wide cache of oracle Remez results (multiprecision)."""
    from oracle.remez import remez
    return remez(alpha, k, m=m, beta=beta)


@pytest.fixture(scope="session")
def bura():
    return oracle_bura
