"""The library's sinc-quadrature terms (bura_sinc_coefficients, C ABI, CPU only) against the oracle."""

import numpy as np
import pytest

from oracle import quadrature


def _lib():
    import paper_1612_04846_amd as B
    return B


CASES = [(0.25, 9), (0.5, 7), (0.5, 8), (0.75, 6), (0.25, 38), (0.5, 20), (0.75, 13), (0.1, 30), (0.9, 30)]


@pytest.mark.parametrize("alpha,kq", CASES)
@pytest.mark.parametrize("scale", [1.0, 8.0 * 1024 ** 2])
def test_terms_match_oracle(alpha, kq, scale):
    B = _lib()
    kp = B.sinc_kprime(alpha, kq)
    assert kp == pytest.approx(quadrature.sinc_kprime(alpha, kq), rel=1e-15)
    w, s = B.bura_sinc_coefficients(alpha, kp, scale)
    wo, so = quadrature.sinc_terms(alpha, kp, scale)
    assert len(w) == len(wo) == quadrature.systems(alpha, kq)
    assert np.allclose(w, wo, rtol=1e-13, atol=0) and np.allclose(s, so, rtol=1e-13, atol=0)


def test_term_count_beyond_capacity_and_bad_arguments():
    B = _lib()
    w, s = B.bura_sinc_coefficients(0.5, 0.2)       # 249 terms, more than one plan holds
    assert len(w) == 249
    for bad in [(0.0, 0.5, 1.0), (1.0, 0.5, 1.0), (0.5, 0.0, 1.0), (0.5, 0.5, -1.0)]:
        with pytest.raises(B.BuraError):
            B.bura_sinc_coefficients(*bad)
