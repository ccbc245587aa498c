"""Pins of the zero-pole product form (remark on the product form in Section 2.2)."""

import mpmath as mp
import numpy as np
import pytest

import synth
from conftest import oracle_bura
from oracle import product, spectral


@pytest.mark.parametrize("alpha,k", [(0.25, 5), (0.5, 5), (0.75, 5), (0.5, 7)])
def test_zeros_interlace_and_constant(alpha, k):
    """Lemma 2.5: k real negative zeros interlacing with the poles; r vanishes there;
    C equals the sum of the partial-fraction weights (r(t)/t ~ C/t at infinity)."""
    b = oracle_bura(alpha, k)
    z, C = product.zeros_and_constant(b)
    d = b.d[1:]
    assert len(z) == k
    assert z[0] < 0
    for j in range(k):
        assert z[j] > d[j]
        if j + 1 < k:
            assert d[j] > z[j + 1]
    with mp.workdps(b.dps):
        for zj in z:
            # relative to the size of r near zeta_j (the numerator is tiny there)
            assert abs(b.r(zj)) <= mp.mpf(10) ** (-20) * abs(b.r(zj / 2))
        assert abs(C - mp.fsum(b.c)) <= mp.mpf(10) ** (-25) * abs(C)


@pytest.mark.parametrize("alpha,k", [(0.25, 5), (0.75, 7)])
def test_product_equals_partial_fractions(alpha, k):
    """The two evaluations of r(A) A^-1 f agree (they are one rational function)."""
    b = oracle_bura(alpha, k)
    z, C = product.zeros_and_constant(b)
    F = synth.normal_rhs(47, 2, nrhs=2, tag=41)
    Up = product.product_spectral(F, 2, C, z, b.d)
    Ur = spectral.bura_spectral(F, 2, b.c_f64, b.d_f64)
    assert np.linalg.norm(Up - Ur) <= 1e-12 * np.linalg.norm(Ur)
