"""Error measures.  TEST INFRASTRUCTURE.

* rel_err: ||u - u_ref||_2 / ||u_ref||_2 per right-hand side (max over the batch),
  the relative l2 error used in Section 5.3.
* Lemma 2.1, eq. (12): ||u_r - u||_{A^gamma} <= E ||f||_{A^(gamma - 2 beta)}; the
  bound helpers evaluate both sides with the spectral norms of ``spectral``.
"""

from __future__ import annotations

import numpy as np

from . import spectral


def rel_err(u: np.ndarray, ref: np.ndarray) -> float:
    nb = u.shape[0]
    a = u.reshape(nb, -1)
    b = ref.reshape(nb, -1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


def lemma_bound_sides(F, U_r, dim, alpha, E, gamma, beta=1):
    """(lhs, rhs) of eq. (12) per right-hand side, for the constant-coefficient grid."""
    U = spectral.exact_fractional(F, dim, alpha)
    lhs = spectral.energy_norm(U_r - U, dim, gamma)
    rhs = E * spectral.energy_norm(F, dim, gamma - 2 * beta)
    return lhs, rhs
