"""Multi-step BURA (Section 4.4).  TEST INFRASTRUCTURE.

A^-alpha f = A^-alpha_n( ... A^-alpha_2(A^-alpha_1 f)) with sum_i alpha_i = alpha;
each factor is replaced by its 1-BURA, u_i = r_{alpha_i}(A) A^-1 u_{i-1}
(eq. (16) with u_0 = f), applied in the order the steps are given.  The
error of the composition over an eigenvector Psi with eigenvalue lambda is
|lambda prod_i (r_i(lambda)/lambda) - lambda^(1-alpha)| in the ratio
||u_n - u||_A / ||f||_A^-1 of eq. (12) (Lemma 2.1) with gamma = 1 (the quantity of
eq. (28)).
"""

from __future__ import annotations

import numpy as np

from . import shifted, spectral


def multistep_spectral(F: np.ndarray, dim: int, steps) -> np.ndarray:
    """Steps = [(c, d), ...] in application order; constant-coefficient grid, sine eigenbasis."""
    U = np.asarray(F, dtype=np.float64)
    for c, d in steps:
        U = spectral.bura_spectral(U, dim, c, d)
    return U


def multistep_by_solves(A, steps, F: np.ndarray) -> np.ndarray:
    """The same steps by k+1 sparse direct shifted solves each (any coefficients)."""
    U = np.asarray(F, dtype=np.float64)
    for c, d in steps:
        U = shifted.bura_by_solves(A, c, d, U)
    return U


def eigvec_errors_1d(N: int, steps, alpha: float) -> tuple[float, float]:
    """Mean and max over the N eigenvectors of the 1D matrix tridiag(-1/4, 1/2, -1/4)
    (Section 5.1: eigenvalues sin^2(i pi/(2(N+1)))) of the gamma = 1 error ratio."""
    i = np.arange(1, N + 1, dtype=np.float64)
    lam = np.sin(i * np.pi / (2 * (N + 1))) ** 2
    R = np.ones_like(lam)
    for c, d in steps:
        R = R * spectral.rho(lam, c, d)
    e = np.abs(lam * R - lam ** (1.0 - alpha))
    return float(e.mean()), float(e.max())


def two_step_bound(E1: float, E2: float, alpha1: float, alpha2: float, kappa: float) -> float:
    """Right-hand side of eq. (29)."""
    return E2 * kappa ** alpha1 + E1 * kappa ** alpha2 + E1 * E2 * kappa
