"""Seeded synthetic inputs shared by the HIP library's tests/benchmark and the oracle.

This module only draws random numbers and samples simple closed-form
functions on grids.  It contains none of the BURA method's arithmetic (no
operator, no rational approximation, no solve), so that the two independent
implementations can be fed identical inputs.

Layout convention for every grid array: interior nodes only, lexicographic
order with x fastest, i.e. numpy shape (n,)*dim in C order with the last axis
x; a batch of right-hand sides prepends one axis.  All arrays are float64.

Workloads mirror the paper's experiments (Section 5): the scaled five-point
Laplacian on the unit square with h = 1/(n+1) (Section 5.3), its 7-point 3D
analogue, random right-hand sides, sums of eigenmodes and the checkerboard
right-hand side of eq. (32).
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List

import numpy as np

SEED_BASE = 161204846


def rng(tag: int) -> np.random.Generator:
    """Generator for workload ``tag`` (seed = 161204846 + tag)."""
    return np.random.default_rng(SEED_BASE + int(tag))


def grid_shape(n: int, dim: int):
    return (n,) * dim


def uniform_rhs(n: int, dim: int, nrhs: int = 1, tag: int = 1) -> np.ndarray:
    """i.i.d. U[-1,1] right-hand sides, shape (nrhs, n, ..., n)."""
    return rng(tag).uniform(-1.0, 1.0, size=(nrhs,) + grid_shape(n, dim))


def normal_rhs(n: int, dim: int, nrhs: int = 1, tag: int = 2) -> np.ndarray:
    """i.i.d. N(0,1) right-hand sides, shape (nrhs, n, ..., n)."""
    return rng(tag).standard_normal(size=(nrhs,) + grid_shape(n, dim))


def sine_mode(n: int, idx) -> np.ndarray:
    """Grid function prod_a sin(i_a * pi * x_a) at x_a = j/(n+1), j = 1..n.

    ``idx`` lists the mode numbers (one per axis, slowest axis first).
    """
    dim = len(idx)
    j = np.arange(1, n + 1, dtype=np.float64)
    out = np.ones(grid_shape(n, dim))
    for axis, i in enumerate(idx):
        v = np.sin(i * math.pi * j / (n + 1))
        shp = [1] * dim
        shp[axis] = n
        out = out * v.reshape(shp)
    return out


def sine_modes_rhs(n: int, dim: int, nmodes: int = 32, noise: float = 1e-3, tag: int = 3,
                   nrhs: int = 1) -> np.ndarray:
    """Sum of ``nmodes`` random-amplitude sine modes plus uniform noise.

    Mode numbers are drawn uniformly from {1..n}^dim without repetition,
    amplitudes from U[-1,1]; ``noise`` * U[-1,1] is added i.i.d. per node.
    """
    g = rng(tag)
    out = np.zeros((nrhs,) + grid_shape(n, dim))
    for r in range(nrhs):
        seen = set()
        while len(seen) < nmodes:
            seen.add(tuple(int(v) for v in g.integers(1, n + 1, size=dim)))
        for idx in sorted(seen):
            out[r] += g.uniform(-1.0, 1.0) * sine_mode(n, idx)
        out[r] += noise * g.uniform(-1.0, 1.0, size=grid_shape(n, dim))
    return out


def checkerboard_rhs(n: int) -> np.ndarray:
    """The right-hand side of eq. (32) on the (n x n) interior grid of the unit square.

    f = 1 where (x-1/2)(y-1/2) > 0 and -1 otherwise (so -1 on the lines x = 1/2
    and y = 1/2).
    """
    x = np.arange(1, n + 1, dtype=np.float64) / (n + 1)
    X = x.reshape(1, n)
    Y = x.reshape(n, 1)
    return np.where((X - 0.5) * (Y - 0.5) > 0, 1.0, -1.0)[None]


def gaussian_field(n: int, dim: int, corr_len: float = 0.1, sigma: float = 1.0,
                   tag: int = 4) -> np.ndarray:
    """Stationary Gaussian field g on the (n+2)^dim node lattice (boundary included).

    Squared-exponential covariance sigma^2 exp(-r^2 / (2 corr_len^2)) sampled by
    circulant embedding on a periodic grid padded to at least twice the
    domain plus 4 correlation lengths; negative embedding eigenvalues are
    clipped to zero.  Returns an array of shape (n+2,)*dim.
    """
    m = n + 2
    h = 1.0 / (n + 1)
    pad = int(math.ceil(4 * corr_len / h))
    M = 1
    while M < 2 * (m + pad):
        M *= 2
    k = np.arange(M)
    dist = np.minimum(k, M - k) * h
    r2 = np.zeros((M,) * dim)
    for axis in range(dim):
        shp = [1] * dim
        shp[axis] = M
        r2 = r2 + (dist ** 2).reshape(shp)
    cov = sigma ** 2 * np.exp(-r2 / (2 * corr_len ** 2))
    lam = np.fft.fftn(cov).real
    lam = np.clip(lam, 0.0, None)
    g = rng(tag)
    z = g.standard_normal((M,) * dim) + 1j * g.standard_normal((M,) * dim)
    field = np.fft.fftn(np.sqrt(lam / lam.size) * z).real
    sl = tuple(slice(0, m) for _ in range(dim))
    return np.ascontiguousarray(field[sl])


def lognormal_coefficient(n: int, dim: int, corr_len: float = 0.1, sigma: float = 1.0,
                          tag: int = 4) -> np.ndarray:
    """Nodal diffusion coefficient a = exp(g) on the (n+2)^dim lattice."""
    return np.exp(gaussian_field(n, dim, corr_len, sigma, tag))


# ----------------------------------------------------------------------------
# serving workload: a seeded Poisson request stream
# ----------------------------------------------------------------------------

SERVING_SHAPES = [(2, 127), (2, 255), (2, 511), (2, 1023), (3, 63), (3, 127), (3, 255)]
SERVING_ALPHAS = [0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9]


@dataclass
class Request:
    arrival: float     # seconds after stream start
    dim: int
    n: int
    alpha: float
    target: float      # requested accuracy 10^-v, v ~ U[6, 9]
    k: int             # 5 + round(7 (v - 6) / 3)
    rhs_tag: int       # seed tag of its N(0,1) right-hand side


def request_stream(count: int, rate_hz: float, tag: int = 5, shapes=None, alphas=None) -> List[Request]:
    """``count`` requests with exponential inter-arrival times of mean 1/rate_hz."""
    g = rng(tag)
    shapes = SERVING_SHAPES if shapes is None else shapes
    alphas = SERVING_ALPHAS if alphas is None else alphas
    t = 0.0
    out = []
    for i in range(count):
        t += g.exponential(1.0 / rate_hz)
        dim, n = shapes[int(g.integers(0, len(shapes)))]
        alpha = float(alphas[int(g.integers(0, len(alphas)))])
        v = float(g.uniform(6.0, 9.0))
        k = 5 + int(round(7 * (v - 6.0) / 3.0))
        out.append(Request(t, dim, n, alpha, 10.0 ** (-v), k, 1000 + i))
    return out
