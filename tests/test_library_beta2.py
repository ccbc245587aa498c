"""The library's 2-BURA (bura_coefficients with beta = 2, C ABI, CPU only) against the oracle and Tables 9-10."""

import json

import pytest

from conftest import golden_path
from oracle import remez


def _lib():
    import paper_1612_04846_amd as B
    return B


@pytest.mark.parametrize("alpha,k", [(0.25, 4), (0.5, 4), (0.75, 4), (0.5, 6), (0.1, 6), (0.9, 5)])
def test_beta2_matches_oracle(alpha, k):
    B = _lib()
    c, d, E = B.bura_coefficients(alpha, k, beta=2)
    o = remez.remez(alpha, k, m=k + 1, beta=2)
    assert len(c) == k + 2 and len(d) == k + 1
    assert c[0] == pytest.approx(float(o.c0[0]), rel=1e-10)
    assert c[k + 1] == pytest.approx(float(o.c0[1]), rel=1e-10)
    assert c[1:k + 1] == pytest.approx([float(x) for x in o.c[1:]], rel=1e-10)
    assert d[1:] == pytest.approx([float(x) for x in o.d[1:]], rel=1e-10)
    assert E == pytest.approx(abs(float(o.E)), rel=1e-10)


def test_beta2_tables9_10():
    """The library's coefficients against the printed tables directly."""
    B = _lib()
    g = json.load(open(golden_path("tables9_10_beta2_coefficients.json")))
    for mk, byalpha in g["tables"].items():
        k = int(mk.split(",")[1])
        for a, t in byalpha.items():
            c, d, E = B.bura_coefficients(float(a), k, beta=2)
            assert c[0] == pytest.approx(t["c01"], rel=2e-5)
            assert c[k + 1] == pytest.approx(t["c02"], rel=2e-4)
            assert c[1:k + 1] == pytest.approx(t["c"], rel=2e-5)
            assert d[1:] == pytest.approx(t["d"], rel=2e-5)
