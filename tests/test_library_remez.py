"""The library's host Remez (bura_coefficients, C ABI, CPU only) against the oracle and the paper.

The library computes the BURA in __float128 with a barycentric representation;
the oracle in mpmath with the Chebyshev form of eq. (18).  Agreement of the
two independent computations, plus equioscillation of the library's own
r(t) = t sum_j c_j/(t - d_j) evaluated in multiprecision, pins the a0 step.
"""

import json
import os

import mpmath as mp
import pytest

from conftest import golden_path

GOLD = golden_path("oracle_bura_coefficients.json")


def _lib():
    import paper_1612_04846_amd as B
    return B


def _gold():
    if not os.path.exists(GOLD):
        pytest.skip("oracle coefficient file not generated")
    return json.load(open(GOLD))


def _pairs():
    if not os.path.exists(GOLD):
        return []
    d = json.load(open(GOLD))
    out = []
    for key, rec in d.items():
        if key.startswith("_") or "error" in rec:
            continue
        a, k = key.split(",")
        out.append((float(a), int(k)))
    return sorted(out)


@pytest.mark.parametrize("alpha,k", _pairs())
def test_library_matches_oracle(alpha, k):
    rec = _gold()[f"{alpha:.2f},{k}"]
    c, d, E = _lib().bura_coefficients(alpha, k)
    assert abs(E - float(rec["E"])) <= 1e-11 * float(rec["E"])
    for got, ref in zip(c, rec["c"]):
        assert abs(got - float(ref)) <= 1e-11 * abs(float(ref)), (got, ref)
    for got, ref in zip(d[1:], rec["d"][1:]):
        assert abs(got - float(ref)) <= 1e-11 * abs(float(ref)), (got, ref)
    assert d[0] == 0.0


@pytest.mark.parametrize("alpha,k", [(0.5, 5), (0.25, 9), (0.75, 9), (0.1, 12), (0.9, 12), (0.9, 5), (0.6, 7)])
def test_library_equioscillation(alpha, k):
    """Definition 2.1 / Lemma 2.5 on the library's own double-precision output."""
    c, d, E = _lib().bura_coefficients(alpha, k)
    assert c[0] == pytest.approx(E, rel=1e-14)                       # eq. (23)
    assert all(x > 0 for x in c) and all(d[j] > d[j + 1] for j in range(k))
    with mp.workdps(40):
        cm = [mp.mpf(x) for x in c]
        dm = [mp.mpf(x) for x in d]
        g = 1 - mp.mpf(alpha)

        def err(t):
            r = cm[0] + mp.fsum(cm[j] * t / (t - dm[j]) for j in range(1, k + 1))
            return t ** g - r

        # dense grid in log t and in t: nowhere larger than E (up to coefficient rounding)
        grid = [mp.mpf(10) ** (-x / mp.mpf(25)) for x in range(0, 25 * 40)] + [mp.mpf(i) / 400 for i in range(401)]
        vals = [err(t) for t in grid]
        worst = max(abs(v) for v in vals)
        assert worst <= E * (1 + 1e-6)
        # and the error reaches -E at t = 0 and +-E at t = 1 with 2k+1 sign changes in between
        assert err(mp.mpf(0)) == pytest.approx(-E, rel=1e-12)
        assert abs(err(mp.mpf(1))) == pytest.approx(E, rel=1e-6)
        signs = [v > 0 for v in sorted(zip(grid, vals))[::1] for v in [v[1]]]
        changes = sum(1 for a, b in zip(signs, signs[1:]) if a != b)
        assert changes >= 2 * k + 1


@pytest.mark.parametrize("alpha,col", [(0.25, 1), (0.5, 1), (0.25, 3), (0.5, 3), (0.75, 3)])
def test_library_against_table1(alpha, col):
    t1 = json.load(open(golden_path("table1_bura_errors.json")))
    row = [r for r in t1["rows"] if r[0] == alpha][0]
    k = {1: 5, 2: 6, 3: 7}[col]
    _, _, E = _lib().bura_coefficients(alpha, k)
    tol = 1e-2 if alpha == 0.75 else 2e-4
    assert abs(E - row[col]) <= tol * row[col]
