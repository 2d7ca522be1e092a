"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the oracle.

This module only draws random numbers and arranges them; it holds none of the
factorization's arithmetic.  All matrices are float64, column-major (numpy
Fortran order), optionally with a leading dimension ``lda > n`` whose padding
rows hold a NaN sentinel so that stray writes or reads show up.

Workloads (the paper evaluates square matrices with uniformly distributed
random entries, Sec. 6.1):

* ``uniform``   -- i.i.d. uniform[-1, 1)
* ``dominant``  -- uniform[-1, 1) with each diagonal entry replaced by the sum of
                   the absolute values of its row (old diagonal included)
* ``planted``   -- A = P L U from known factors: L unit lower with entries
                   uniform[-a, a), U upper with diagonal uniform[1, 2) and
                   strictly-upper entries uniform[-1, 1)/sqrt(n), and a seeded
                   row permutation: row ``perm[i]`` of A is row i of L U.

Random streams: numpy's Philox bit generator keyed by (seed, stream id);
stream ids 0 = A, 1 = right-hand sides, 2 = permutation, 3 = L, 4 = U.
"""
from __future__ import annotations

import numpy as np

STREAM_A, STREAM_B, STREAM_PERM, STREAM_L, STREAM_U = 0, 1, 2, 3, 4


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[int(seed), int(stream)]))


def _alloc(n: int, ncols: int, lda: int | None) -> np.ndarray:
    lda = n if lda is None else int(lda)
    if lda < max(1, n):
        raise ValueError("lda must be >= max(1, n)")
    buf = np.empty((lda, ncols), dtype=np.float64, order="F")
    if lda > n:
        buf[n:, :] = np.nan
    return buf[:n, :]


def _fill_uniform(out: np.ndarray, g: np.random.Generator, lo=-1.0, hi=1.0) -> None:
    """out[:] = uniform[lo, hi) drawn column by column (53-bit mantissas)."""
    n, ncols = out.shape
    step = max(1, (1 << 24) // max(n, 1))
    for j0 in range(0, ncols, step):
        j1 = min(ncols, j0 + step)
        u = g.random((j1 - j0, n))            # [0,1) doubles, k * 2**-53
        u *= (hi - lo)
        u += lo
        out[:, j0:j1] = u.T


def uniform(n: int, seed: int = 1, lda: int | None = None, stream: int = STREAM_A) -> np.ndarray:
    A = _alloc(n, n, lda)
    _fill_uniform(A, rng(seed, stream))
    return A


def rhs(n: int, seed: int = 1, nrhs: int = 1, ldb: int | None = None) -> np.ndarray:
    B = _alloc(n, nrhs, ldb)
    _fill_uniform(B, rng(seed, STREAM_B))
    return B


def dominant(n: int, seed: int = 1, lda: int | None = None) -> np.ndarray:
    A = uniform(n, seed, lda)
    s = np.zeros(n)
    for j in range(n):                        # row sums of |a_ij|, column by column
        s += np.abs(A[:, j])
    A[np.arange(n), np.arange(n)] = s
    return A


def spd(n: int, seed: int = 1, lda: int | None = None) -> np.ndarray:
    """Symmetric positive definite workload for Cholesky: the symmetric part
    (B + B^T)/2 of a uniform[-1,1) matrix B, with each diagonal entry set to
    its row's absolute sum (strictly diagonally dominant, positive diagonal)."""
    B = uniform(n, seed, lda)
    A = B[:n, :n]
    A[:] = (A + A.T) / 2.0
    s = np.zeros(n)
    for j in range(n):
        s += np.abs(A[:, j])
    A[np.arange(n), np.arange(n)] = s
    return B


def planted_factors(n: int, seed: int = 1, a_l: float = 0.1):
    """Return (L, U, perm) of the planted workload (dense float64 arrays)."""
    gl, gu, gp = rng(seed, STREAM_L), rng(seed, STREAM_U), rng(seed, STREAM_PERM)
    L = np.zeros((n, n), order="F")
    _fill_uniform(L, gl, -a_l, a_l)
    L = np.tril(L, -1)
    np.fill_diagonal(L, 1.0)
    U = np.zeros((n, n), order="F")
    _fill_uniform(U, gu, -1.0, 1.0)
    U = np.triu(U, 1) / np.sqrt(max(n, 1))
    U[np.arange(n), np.arange(n)] = 1.0 + gu.random(n)
    perm = gp.permutation(n)
    return L, U, perm


def planted(n: int, seed: int = 1, a_l: float = 0.1, lda: int | None = None, matmul=None):
    """A with row perm[i] equal to row i of L @ U; returns (A, L, U, perm).

    ``matmul`` computes the product of the two factors (numpy by default; a
    caller may pass a faster library routine for large n).
    """
    L, U, perm = planted_factors(n, seed, a_l)
    prod = (matmul or np.matmul)(L, U)
    A = _alloc(n, n, lda)
    A[perm, :] = prod
    return A, L, U, perm
