"""Pins of the multi-step BURA oracle (Section 4.4)."""

import json

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from conftest import golden_path, oracle_coeffs
from oracle import multistep, operators, spectral


def _steps(alphas, k):
    out = []
    for a in alphas:
        b = oracle_coeffs(a, k)
        out.append((b.c_f64, b.d_f64))
    return out


@pytest.mark.parametrize("k", [5, 7])
def test_tables13_14_eigenvector_columns(k):
    """Every eigenvector column of Tables 13 and 14 (mean and max over the
    eigenvectors, three setups, all printed grid sizes) to its printed digits."""
    g = json.load(open(golden_path("tables13_14_multistep_eigvec.json")))
    for h, row in g[f"k{k}"].items():
        for s, alphas in enumerate(g["setups"]):
            mean, mx = multistep.eigvec_errors_1d(int(h), _steps(alphas, k), sum(alphas))
            assert mean == pytest.approx(row["mean"][s], rel=2e-4), (k, h, alphas)
            assert mx == pytest.approx(row["max"][s], rel=2e-4), (k, h, alphas)


def test_two_step_error_within_bound_and_order_free():
    """eq. (29) bounds the A-norm error over every eigenvector, and
    the product form makes the order of the steps irrelevant (up to rounding)."""
    n = 31
    F = synth.normal_rhs(n, 2, nrhs=2, tag=31)
    lam = spectral.eigenvalues(n, 2)
    kappa = lam.max() / lam.min()
    a1, a2, k = 0.5, 0.25, 5
    s12 = _steps([a1, a2], k)
    s21 = _steps([a2, a1], k)
    U12 = multistep.multistep_spectral(F, 2, s12)
    U21 = multistep.multistep_spectral(F, 2, s21)
    assert np.allclose(U12, U21, rtol=1e-12, atol=1e-12 * np.abs(U12).max())
    Ue = spectral.exact_fractional(F, 2, a1 + a2)
    E1, E2 = float(oracle_coeffs(a1, k).E), float(oracle_coeffs(a2, k).E)
    bound = multistep.two_step_bound(E1, E2, a1, a2, kappa)
    for r in range(2):
        num = spectral.energy_norm(U12[r] - Ue[r], 2, 1.0)
        den = spectral.energy_norm(F[r], 2, -1.0)
        assert num <= bound * den


def test_solves_match_spectral_variable_coefficient_reduces():
    """Sparse shifted solves reproduce the eigenbasis evaluation (constant
    coefficients), and a one-step program is the plain BURA."""
    n = 15
    F = synth.normal_rhs(n, 2, nrhs=1, tag=32)
    A, _ = operators.scaled_operator(n, 2)
    st = _steps([0.25, 0.25, 0.25], 5)
    Us = multistep.multistep_by_solves(A, st, F.reshape(1, -1)).reshape(F.shape)
    Up = multistep.multistep_spectral(F, 2, st)
    assert np.allclose(Us, Up, rtol=1e-11, atol=1e-13)
    one = multistep.multistep_spectral(F, 2, st[:1])
    assert np.array_equal(one, spectral.bura_spectral(F, 2, *st[0]))
    assert sp.issparse(A)
