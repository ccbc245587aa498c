"""O3: the BURA result by k+1 shifted sparse solves, eq. (16).  TEST INFRASTRUCTURE.

u_r = sum_{j=0..k} c_j (A - d_j I)^-1 f  (Section 2.2, Steps 1-3), each system
solved independently -- by a sparse direct factorisation (SuperLU) or, for
large 3D grids, by plain conjugate gradients to a tight relative residual --
and summed in FP64 in the order j = 0..k.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def shifted_factor(A: sp.spmatrix, shift: float):
    """SuperLU factorisation of A + shift I (its .solve applies the inverse)."""
    N = A.shape[0]
    return spla.splu((A + shift * sp.identity(N, format="csr")).tocsc())


def shifted_solve_direct(A: sp.spmatrix, shift: float, F: np.ndarray) -> np.ndarray:
    """(A + shift I)^-1 F for a batch F of shape (nrhs, N) by SuperLU."""
    N = A.shape[0]
    lu = shifted_factor(A, shift)
    return lu.solve(np.ascontiguousarray(F.reshape(F.shape[0], N).T)).T


def cg(A: sp.spmatrix, b: np.ndarray, shift: float = 0.0, rtol: float = 1e-14, maxiter: int = 100000):
    """Plain FP64 conjugate gradients for (A + shift I) x = b (textbook, no preconditioner)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(r @ r)
    nb = float(np.sqrt(b @ b))
    it = 0
    while np.sqrt(rr) > rtol * nb and it < maxiter:
        q = A @ p + shift * p
        a = rr / float(p @ q)
        x += a * p
        r -= a * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def bura_by_solves(A: sp.spmatrix, c, d, F: np.ndarray, method: str = "direct",
                   rtol: float = 1e-14) -> np.ndarray:
    """u_r for every right-hand side in F (shape (nrhs, n, ..., n))."""
    shape = F.shape
    N = A.shape[0]
    Fm = F.reshape(shape[0], N)
    U = np.zeros_like(Fm)
    for cj, dj in zip(c, d):
        if method == "direct":
            W = shifted_solve_direct(A, -dj, Fm)
        else:
            W = np.stack([cg(A, Fm[r], -dj, rtol)[0] for r in range(shape[0])])
        U = U + cj * W
    return U.reshape(shape)


def residual_norms(A: sp.spmatrix, shift: float, X: np.ndarray, F: np.ndarray) -> np.ndarray:
    """||F - (A + shift) X||_2 / ||F||_2 per right-hand side."""
    N = A.shape[0]
    Xm = X.reshape(X.shape[0], N)
    Fm = F.reshape(F.shape[0], N)
    R = Fm - (A @ Xm.T).T - shift * Xm
    return np.linalg.norm(R, axis=1) / np.linalg.norm(Fm, axis=1)
