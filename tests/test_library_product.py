"""The library's zeros and leading constant (bura_zeros, C ABI, CPU only) against the oracle."""

import mpmath as mp
import pytest

from conftest import oracle_bura
from oracle import product


def _lib():
    import paper_1612_04846_amd as B
    return B


@pytest.mark.parametrize("alpha,k", [(0.25, 5), (0.5, 5), (0.75, 5), (0.5, 7), (0.25, 9)])
def test_zeros_match_oracle(alpha, k):
    B = _lib()
    z, C = B.bura_zeros(alpha, k)
    zo, Co = product.zeros_and_constant(oracle_bura(alpha, k))
    assert len(z) == k
    for a, b in zip(z, zo):
        assert a == pytest.approx(float(b), rel=1e-10)
    assert C == pytest.approx(float(Co), rel=1e-11)


@pytest.mark.parametrize("alpha,k", [(0.9, 12), (0.1, 12), (0.75, 16)])
def test_zeros_interlace_where_the_oracle_cannot_go(alpha, k):
    """Lemma 2.5 on the library's own zeros and poles, and C = sum of the weights."""
    B = _lib()
    z, C = B.bura_zeros(alpha, k)
    c, d, E = B.bura_coefficients(alpha, k)
    assert z[0] < 0
    for j in range(k):
        assert z[j] > d[j + 1]
        if j + 1 < k:
            assert d[j + 1] > z[j + 1]
    assert C == pytest.approx(float(mp.fsum(c)), rel=1e-11)
