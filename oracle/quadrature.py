"""Sinc quadrature u_Q of Bonito and Pasciak, the comparison method of Section 5.3.  TEST INFRASTRUCTURE.

Section 5.3 (the displayed formula for u_Q after eq. (32)) approximates
A~^-alpha f~ for the unscaled grid matrix A~ by

    u_Q = (2 k' sin(pi alpha) / pi) * sum_{l=-m}^{M} exp(2 (alpha - 1) l k') (exp(-2 l k') I + A~)^-1 f~,
    m = ceil(pi^2 / (4 alpha k'^2)),   M = ceil(pi^2 / (4 (1 - alpha) k'^2)),

with a free step k' > 0.  The same section relates k' to the nominal number
of systems k_Q = pi^2 / (4 alpha (1 - alpha) k'^2) and restricts itself to
integer k_Q.  This is the trapezoidal rule with step k' in y applied to the
integral lambda^-alpha = (2 sin(pi alpha)/pi) int exp(2(alpha-1)y) / (exp(-2y) + lambda) dy,
which is what the tests pin it against.

Reading (the paper is silent on rounding): when k' comes from an integer
k_Q, pi^2/(4 alpha k'^2) = (1 - alpha) k_Q exactly, so the ceilings are of
exact rationals; floating point values within 1e-9 (relative) of an integer
are taken as that integer before the ceiling.

The operator the rule is applied to matters (the rule is not scale
invariant).  ``sinc_terms(alpha, kprime, scale)`` applies it to scale * A for
the scaled A of eq. (algebraic) and returns (w, s) with
sum_j w_j (A + s_j I)^-1 f ~= A^-alpha f, i.e.
w_l = scale^(alpha-1) * (2 k' sin(pi alpha)/pi) exp(2(alpha-1) l k'), s_l = exp(-2 l k') / scale.
With scale = Lambda this is the paper's u_Q (applied to A~ = Lambda A)
multiplied by Lambda^alpha.
"""

from __future__ import annotations

import math

import mpmath as mp
import numpy as np

from . import spectral

_DPS = 40


def sinc_kprime(alpha: float, kq: float) -> float:
    """k' with pi^2 / (4 alpha (1 - alpha) k'^2) = k_Q (Section 5.3)."""
    with mp.workdps(_DPS):
        return float(mp.pi / (2 * mp.sqrt(mp.mpf(alpha) * (1 - mp.mpf(alpha)) * kq)))


def _ceil_reading(x) -> int:
    r = mp.nint(x)
    if abs(x - r) <= mp.mpf("1e-9") * abs(x):
        return int(r)
    return int(mp.ceil(x))


def sinc_counts(alpha: float, kprime: float) -> tuple[int, int]:
    """(m, M) of Section 5.3's formula; the rule has m + M + 1 terms."""
    with mp.workdps(_DPS):
        a, kp = mp.mpf(alpha), mp.mpf(kprime)
        m = _ceil_reading(mp.pi ** 2 / (4 * a * kp ** 2))
        M = _ceil_reading(mp.pi ** 2 / (4 * (1 - a) * kp ** 2))
    return m, M


def sinc_terms(alpha: float, kprime: float, scale: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """Weights w and shifts s (l = -m .. M, in that order) for the scaled operator A.

    sum_l w_l (A + s_l I)^-1 f equals scale^alpha times the rule applied to scale*A."""
    m, M = sinc_counts(alpha, kprime)
    w, s = [], []
    with mp.workdps(_DPS):
        a, kp, sc = mp.mpf(alpha), mp.mpf(kprime), mp.mpf(scale)
        pref = 2 * kp * mp.sin(mp.pi * a) / mp.pi
        for l in range(-m, M + 1):
            w.append(float(sc ** (a - 1) * pref * mp.exp(2 * (a - 1) * l * kp)))
            s.append(float(mp.exp(-2 * l * kp) / sc))
    return np.array(w), np.array(s)


def sinc_scalar(lam, alpha: float, kprime: float) -> np.ndarray:
    """The rule applied to a scalar (or array) lambda > 0: ~ lambda^-alpha."""
    w, s = sinc_terms(alpha, kprime, 1.0)
    lam = np.asarray(lam, dtype=np.float64)
    out = np.zeros_like(lam)
    for wj, sj in zip(w, s):
        out = out + wj / (lam + sj)
    return out


def sinc_spectral(F: np.ndarray, dim: int, alpha: float, kprime: float, scale: float) -> np.ndarray:
    """sum_l w_l (A + s_l I)^-1 F for the constant-coefficient scaled grid operator, in its sine eigenbasis."""
    w, s = sinc_terms(alpha, kprime, scale)

    def phi(lam):
        out = np.zeros_like(lam)
        for wj, sj in zip(w, s):
            out = out + wj / (lam + sj)
        return out

    return spectral.apply_function(F, dim, phi)


def systems(alpha: float, kq: int) -> int:
    """Number of shifted systems of the rule with k' taken from an integer k_Q."""
    m, M = sinc_counts(alpha, sinc_kprime(alpha, kq))
    return m + M + 1


def kq_from_kprime(alpha: float, kprime: float) -> float:
    return math.pi ** 2 / (4 * alpha * (1 - alpha) * kprime ** 2)
