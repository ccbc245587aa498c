"""Scaled SPD grid operators as scipy.sparse matrices.  TEST INFRASTRUCTURE.

* Section 1.4, eq. (10) and Assumption 1.1: A = A~/Lambda with Lambda an upper
  bound of the spectrum of A~, so that spec(A) lies in (0,1].
* Section 5.3: the five-point Laplacian A~ = h^-2 tridiag(-I, tridiag(-1,4,-1), -I)
  on the unit square, h = 1/(n+1), lexicographic order, scaled to A = h^2 A~/8.
  The 3D 7-point analogue is scaled by h^2/12 (same rule, 4d/h^2 for d = 3).
* Variable coefficients (reading): flux form
      (A~ x)_i = h^-2 sum_faces a_f (x_i - x_nb),  x_nb = 0 on the boundary,
  with a_f = 2 a_i a_nb / (a_i + a_nb) the harmonic mean of the nodal values
  on the (n+2)^d lattice.  Lambda is Gershgorin's bound max_i sum_j |A~_ij|.
* Constant coefficients: Lambda = 4d/h^2, the paper's own scaling, for every
  n.  (Gershgorin's bound equals it for n >= 3; for n <= 2 no node has all its
  neighbours inside and Gershgorin is smaller.  The closed-form eigenbasis of
  `spectral` uses 4d/h^2.)
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _lex_index(n, dim):
    return np.arange(n ** dim).reshape((n,) * dim)


def unscaled_operator(n: int, dim: int, a_nodes: np.ndarray | None = None) -> sp.csr_matrix:
    """A~ for the constant (a_nodes None) or variable coefficient problem."""
    h = 1.0 / (n + 1)
    N = n ** dim
    idx = _lex_index(n, dim)
    diag = np.zeros((n,) * dim)
    rows, cols, vals = [], [], []
    for axis in range(dim):
        # faces between interior node i and i+1 along `axis` (including the
        # faces to the two boundary nodes)
        if a_nodes is None:
            face = np.ones(tuple(n + 1 if ax == axis else n for ax in range(dim)))
        else:
            inner = tuple(slice(1, n + 1) if ax != axis else slice(None) for ax in range(dim))
            aa = a_nodes[inner]                       # (n+2) along axis, n elsewhere
            lo = tuple(slice(0, n + 1) if ax == axis else slice(None) for ax in range(dim))
            hi = tuple(slice(1, n + 2) if ax == axis else slice(None) for ax in range(dim))
            face = 2.0 * aa[lo] * aa[hi] / (aa[lo] + aa[hi])
        # contributions: face j sits between node j-1 and j (node 0 and n+1 are boundary)
        lo_face = tuple(slice(0, n) if ax == axis else slice(None) for ax in range(dim))
        hi_face = tuple(slice(1, n + 1) if ax == axis else slice(None) for ax in range(dim))
        diag += face[lo_face] + face[hi_face]
        # off-diagonal between interior nodes i and i+1 along axis
        src = tuple(slice(0, n - 1) if ax == axis else slice(None) for ax in range(dim))
        dst = tuple(slice(1, n) if ax == axis else slice(None) for ax in range(dim))
        fin = tuple(slice(1, n) if ax == axis else slice(None) for ax in range(dim))
        w = face[fin].ravel()
        r = idx[src].ravel()
        c = idx[dst].ravel()
        rows += [r, c]
        cols += [c, r]
        vals += [-w, -w]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return A / h ** 2


def gershgorin_bound(A: sp.spmatrix) -> float:
    """Lambda = max_i sum_j |A_ij|, an upper bound of the spectrum."""
    return float(np.max(np.asarray(abs(A).sum(axis=1)).ravel()))


def scaled_operator(n: int, dim: int, a_nodes: np.ndarray | None = None):
    """(A, Lambda) with A = A~/Lambda as in eq. (10)."""
    At = unscaled_operator(n, dim, a_nodes)
    lam = 4.0 * dim * (n + 1) ** 2 if a_nodes is None else gershgorin_bound(At)
    return (At / lam).tocsr(), lam
