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


class _Stored:
    """Oracle coefficients read back from tests/golden/oracle_bura_coefficients.json."""

    def __init__(self, rec):
        import mpmath as mp
        self.c = [mp.mpf(x) for x in rec["c"]]
        self.d = [mp.mpf(x) for x in rec["d"]]
        self.E = mp.mpf(rec["E"])
        self.c_f64 = [float(x) for x in rec["c"]]
        self.d_f64 = [float(x) for x in rec["d"]]


@functools.lru_cache(maxsize=None)
def oracle_coeffs(alpha, k):
    """The oracle's (k,k) BURA coefficients: stored file if present, else computed now."""
    import json
    path = os.path.join(GOLDEN, "oracle_bura_coefficients.json")
    if os.path.exists(path):
        rec = json.load(open(path)).get(f"{alpha:.2f},{k}")
        if rec and "error" not in rec:
            return _Stored(rec)
    return oracle_bura(alpha, k)


@pytest.fixture(scope="session")
def bura():
    return oracle_bura
