"""Zero-pole product form of the 1-BURA (remark on the product form in Section 2.2).  TEST INFRASTRUCTURE.

r(t) = C prod_{j=1..k} (t - zeta_j)/(t - d_j) with the zeros zeta_j of the
numerator and the poles d_j of the denominator of r = P/Q (Lemma 2.5: real,
negative, interlacing), C = p_k / q_k.  The remark evaluates
r(A) A^-1 f = C prod_j (A - zeta_j I)(A - d_j I)^-1 A^-1 f factor by factor:
v_0 = A^-1 f, v_j = (A - zeta_j I)(A - d_j I)^-1 v_{j-1}, u = C v_k.
"""

from __future__ import annotations

import mpmath as mp
import numpy as np

from . import spectral
from .remez import Bura, RemezError


def zeros_and_constant(b: Bura):
    """(zeta_1 > ... > zeta_k, C) from the monomial numerator of the oracle's BURA."""
    with mp.workdps(b.dps):
        roots = mp.polyroots(list(reversed(b.p)), maxsteps=400, extraprec=4 * b.dps)
        z = []
        for w in roots:
            if abs(mp.im(w)) > mp.mpf(10) ** (-(b.dps // 3)) * (1 + abs(w)):
                raise RemezError("complex zero")
            z.append(mp.re(w))
        z = sorted(z, reverse=True)
        C = b.p[b.m] / b.q[b.k]
    return z, C


def product_spectral(F: np.ndarray, dim: int, C, zeta, d) -> np.ndarray:
    """The factor-by-factor evaluation on a constant-coefficient grid (sine eigenbasis)."""
    V = spectral.apply_function(np.asarray(F, dtype=np.float64), dim, lambda lam: 1.0 / lam)
    for zj, dj in zip(zeta, d[1:]):
        zj, dj = float(zj), float(dj)
        V = spectral.apply_function(V, dim, lambda lam, zj=zj, dj=dj: (lam - zj) / (lam - dj))
    return float(C) * V
