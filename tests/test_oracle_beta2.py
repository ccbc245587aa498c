"""Pins of the oracle's 2-BURA (beta = 2, Section 4.1 and eq. (25))."""

import json

import mpmath as mp
import numpy as np
import pytest

import synth
from conftest import golden_path
from oracle import remez, spectral


def _b2(alpha, m, k):
    return remez.remez(alpha, k, m=m, beta=2)


@pytest.mark.parametrize("mk", ["5,4", "7,6"])
@pytest.mark.parametrize("alpha", [0.25, 0.5, 0.75])
def test_tables9_10_coefficients(mk, alpha):
    """Every printed coefficient of Tables 9 and 10 (c_{0,1}, c_{0,2}, c_j, d_j)."""
    g = json.load(open(golden_path("tables9_10_beta2_coefficients.json")))
    t = g["tables"][mk][str(alpha)]
    m, k = (int(x) for x in mk.split(","))
    b = _b2(alpha, m, k)
    assert float(b.c0[0]) == pytest.approx(t["c01"], rel=2e-5)
    assert float(b.c0[1]) == pytest.approx(t["c02"], rel=2e-4)   # printed with 5 digits
    assert [float(x) for x in b.c[1:]] == pytest.approx(t["c"], rel=2e-5)
    assert [float(x) for x in b.d[1:]] == pytest.approx(t["d"], rel=2e-5)


@pytest.mark.parametrize("alpha", [0.25, 0.75])
def test_beta2_identities(alpha):
    """eq. (23): c_{0,2} = P(0)/Q(0) = +-E (negative here, as in the tables); the
    fractions reproduce r(t)/t^2; the 2-BURA equioscillates (m+k+2 points)."""
    b = _b2(alpha, 5, 4)
    with mp.workdps(b.dps):
        assert abs(abs(b.c0[1]) - abs(b.E)) <= mp.mpf(10) ** (-30) * abs(b.E)
        assert b.c0[1] < 0
        for t in [mp.mpf(10) ** (-e) for e in range(0, 9)] + [mp.mpf("0.37"), mp.mpf(3)]:
            frac = b.c0[1] / t ** 2 + b.c0[0] / t + mp.fsum(cj / (t - dj) for cj, dj in zip(b.c[1:], b.d[1:]))
            assert abs(frac - b.r(t) / t ** 2) <= mp.mpf(10) ** (-25) * abs(b.r(t) / t ** 2)
        errs = [b.err(t) for t in b.eta]
        assert len(errs) == 5 + 4 + 2
        for e1, e2 in zip(errs, errs[1:]):
            assert e1 * e2 < 0
            assert abs(abs(e1) - abs(b.E)) <= mp.mpf(10) ** (-12) * abs(b.E)


def test_beta2_spectral_within_lemma_bound():
    """u_r = r(A) A^-2 f approximates A^-alpha f within E ||A^-2 f|| (Lemma 2.1 with beta = 2)."""
    n, alpha = 31, 0.5
    b = _b2(alpha, 5, 4)
    F = synth.normal_rhs(n, 2, nrhs=2, tag=61)
    lam = spectral.eigenvalues(n, 2)
    Ur = spectral.bura_beta_spectral(F, 2, b.c0, b.c, b.d)
    Ue = spectral.exact_fractional(F, 2, alpha)
    A2f = spectral.apply_function(F, 2, lambda l: l ** -2.0)
    for r in range(2):
        assert np.linalg.norm(Ur[r] - Ue[r]) <= abs(float(b.E)) * np.linalg.norm(A2f[r]) * (1 + 1e-9)
    assert np.all(lam > 0)
