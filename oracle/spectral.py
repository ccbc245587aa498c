"""O2: closed-form spectral solutions for the constant-coefficient grids.  TEST INFRASTRUCTURE.

* eq. (9): u = A^-alpha f = W D^-alpha W^T f with orthonormal eigenvectors W.
* Section 5.1 gives, for the scaled 1D matrix tridiag(-1/4, 1/2, -1/4),
  Lambda_i = sin^2(i pi / (2(N+1))) and Psi_i = (sin(i k pi/(N+1)))_k.  The
  scaled d-dimensional operator of Section 5.3 (A = h^2 A~/(4d)) is the
  average of the d one-dimensional ones, so its eigenvalues are
  (1/d) sum_a sin^2(i_a pi/(2(n+1))) and its eigenvectors are tensor products
  of the 1D sines.  The orthonormal sine transform (DST-I, 'ortho') is its own
  inverse, so W^T and W are both one call.
* eq. (16): the BURA result u_r = sum_j c_j (A - d_j I)^-1 f is, in the
  eigenbasis, multiplication by rho(lambda) = sum_j c_j/(lambda - d_j) = r(lambda)/lambda.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def eigenvalues(n: int, dim: int) -> np.ndarray:
    """Eigenvalues of the scaled operator, shape (n,)*dim, axis order matches the grid."""
    i = np.arange(1, n + 1, dtype=np.float64)
    s = np.sin(i * np.pi / (2 * (n + 1))) ** 2
    lam = np.zeros((n,) * dim)
    for axis in range(dim):
        shp = [1] * dim
        shp[axis] = n
        lam = lam + s.reshape(shp)
    return lam / dim


def to_eigenbasis(F: np.ndarray, dim: int) -> np.ndarray:
    """W^T F for a batch F of shape (nrhs, n, ..., n)."""
    axes = tuple(range(F.ndim - dim, F.ndim))
    return sfft.dstn(F, type=1, norm="ortho", axes=axes)


def from_eigenbasis(G: np.ndarray, dim: int) -> np.ndarray:
    axes = tuple(range(G.ndim - dim, G.ndim))
    return sfft.idstn(G, type=1, norm="ortho", axes=axes)


def apply_function(F: np.ndarray, dim: int, phi) -> np.ndarray:
    """W phi(D) W^T F."""
    n = F.shape[-1]
    lam = eigenvalues(n, dim)
    return from_eigenbasis(phi(lam) * to_eigenbasis(F, dim), dim)


def exact_fractional(F: np.ndarray, dim: int, alpha: float) -> np.ndarray:
    """A^-alpha F, eq. (9)."""
    return apply_function(F, dim, lambda lam: lam ** (-alpha))


def rho(lam: np.ndarray, c, d) -> np.ndarray:
    """r(lambda)/lambda = sum_j c_j/(lambda - d_j), summed in j order (eq. (15))."""
    out = np.zeros_like(lam)
    for cj, dj in zip(c, d):
        out = out + cj / (lam - dj)
    return out


def bura_spectral(F: np.ndarray, dim: int, c, d) -> np.ndarray:
    """u_r = sum_j c_j (A - d_j I)^-1 F evaluated exactly in the eigenbasis (eq. (16))."""
    return apply_function(F, dim, lambda lam: rho(lam, c, d))


def shifted_inverse_spectral(F: np.ndarray, dim: int, shift: float) -> np.ndarray:
    """(A + shift I)^-1 F, shift >= 0, for one pole."""
    return apply_function(F, dim, lambda lam: 1.0 / (lam + shift))


def energy_norm(X: np.ndarray, dim: int, gamma: float) -> np.ndarray:
    """||x||_{A^gamma} = sqrt(x^T A^gamma x) per batch entry (notation of Section 1.2)."""
    n = X.shape[-1]
    lam = eigenvalues(n, dim)
    G = to_eigenbasis(X, dim)
    axes = tuple(range(X.ndim - dim, X.ndim))
    return np.sqrt(np.sum(lam ** gamma * G ** 2, axis=axes))


def bura_beta_spectral(F: np.ndarray, dim: int, c0, c, d) -> np.ndarray:
    """eq. (25) in the eigenbasis: u_r = sum_i c0[i-1] A^-i f + sum_{j>=1} c_j (A - d_j I)^-1 f,
    i = 1..beta (c[0], d[0] belong to the pole at 0 and are carried by c0)."""
    def phi(lam):
        out = np.zeros_like(lam)
        for i, ci in enumerate(c0, start=1):
            out = out + float(ci) / lam ** i
        for cj, dj in zip(c[1:], d[1:]):
            out = out + float(cj) / (lam - float(dj))
        return out
    return apply_function(F, dim, phi)
