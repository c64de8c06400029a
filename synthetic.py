"""Seeded synthetic inputs shaped like the paper's workloads.

The paper (Performance evaluation, experimental results) times the product on
randomly generated square matrices of order 5000 and 10000 and motivates A^t A
by least squares and the normal equations (Introduction).  No dataset exists;
these generators stand in for those inputs.

This module holds random-number generation only: none of the A^t A method's
arithmetic lives here.  Both the CPU oracle and the GPU library receive the
arrays it returns; neither imports the other.
"""
from __future__ import annotations

import numpy as np

# Fixed seeds of the standard workloads.
SEED_UNIFORM_SMALL = 0
SEED_INTEGER_SMALL = 1
SEED_SQUARE = 2
SEED_TALL_Z = 3
SEED_TALL_SCALES = 4
SEED_PRECISION = 5
SEED_STREAM = 6
SEED_FACTOR = 7
SEED_REQUEST_BASE = 1000


def uniform(m: int, n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """i.i.d. uniform[-1, 1] entries, row-major m x n (generated in float64)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=(m, n))
    return np.ascontiguousarray(a.astype(dtype, copy=False))


def integer(m: int, n: int, seed: int, lo: int = -3, hi: int = 3, dtype=np.float64) -> np.ndarray:
    """i.i.d. integers uniform in {lo..hi}, stored as floating point."""
    rng = np.random.default_rng(seed)
    a = rng.integers(lo, hi + 1, size=(m, n))
    return np.ascontiguousarray(a.astype(dtype))


def normal(m: int, n: int, seed: int, dtype=np.float64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal(size=(m, n)).astype(dtype, copy=False))


def integer_factor(n: int, seed: int, lo: int = -2, hi: int = 2) -> np.ndarray:
    """Dense n x n lower-triangular integer matrix with diagonal entries drawn
    from {1, 2, 4} and off-diagonal entries uniform in {lo..hi}.  Its Gram
    L L^t has integer entries and a Cholesky factor (L itself) that every
    summation order reaches exactly while partial sums stay below 2^24."""
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(lo, hi + 1, size=(n, n)), -1).astype(np.float64)
    L[np.arange(n), np.arange(n)] = rng.choice([1.0, 2.0, 4.0], size=n)
    return L


def column_scales(n: int, seed: int, lo_exp: float = -3.0, hi_exp: float = 3.0) -> np.ndarray:
    """Log-uniform column scales 10**U(lo_exp, hi_exp)."""
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(lo_exp, hi_exp, size=n)


def tall_scaled(m: int, n: int, seed_z: int = SEED_TALL_Z, seed_s: int = SEED_TALL_SCALES,
                dtype=np.float64) -> np.ndarray:
    """Least-squares shaped input: standard normal entries, columns multiplied by
    log-uniform scales in [1e-3, 1e3] (condition number around 1e6)."""
    z = normal(m, n, seed_z)
    z *= column_scales(n, seed_s)[None, :]
    return np.ascontiguousarray(z.astype(dtype, copy=False))


def hadamard(order: int) -> np.ndarray:
    """Sylvester-Hadamard matrix of a power-of-two order (entries +-1)."""
    if order < 1 or order & (order - 1):
        raise ValueError("order must be a power of two")
    h = np.ones((1, 1))
    while h.shape[0] < order:
        h = np.block([[h, h], [h, -h]])
    return h


def with_lda(a: np.ndarray, lda: int, fill: float = np.nan) -> np.ndarray:
    """Copy a row-major m x n array into a buffer of row stride lda >= n.
    The padding columns hold `fill` so that a reader touching them is caught."""
    m, n = a.shape
    if lda < n:
        raise ValueError("lda must be >= n")
    buf = np.full((m, lda), fill, dtype=a.dtype)
    buf[:, :n] = a
    return buf


def request_stream(count: int, seed: int = SEED_STREAM, rate_per_s: float = 1000.0,
                   m_range=(1024, 65536), n_range=(64, 4096)):
    """Poisson arrivals with log-uniform shapes for the Gram-request stream.

    Returns (arrival_times_s, m, n) arrays: exponential inter-arrival times of
    the given rate, m and n rounded from exp(U(ln lo, ln hi)).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    m = np.rint(np.exp(rng.uniform(np.log(m_range[0]), np.log(m_range[1]), size=count))).astype(np.int64)
    n = np.rint(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]), size=count))).astype(np.int64)
    return t, m, n
