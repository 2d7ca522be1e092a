"""Independent checks that pin the oracle to the mathematics, not to itself.

* ``exact_gepp``: Gaussian elimination with partial pivoting in exact rational
  arithmetic (``fractions.Fraction``; every float64 is an exact dyadic
  rational), pure-Python loops, for tiny n.
* ``leibniz_det``: determinant as the signed sum over all n! permutations.
* ``planted_ipiv``: the pivot sequence partial pivoting must produce on
  A = P L U when every |l_ij| < 1 strictly below the unit diagonal.
* ``top_gap``: smallest relative gap between the two largest candidate
  magnitudes over all elimination steps (flags near-ties).
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def exact_gepp(A: np.ndarray):
    """Return (ipiv, L, U, min_gap) in exact arithmetic; ties -> smallest index."""
    n = A.shape[0]
    M = [[Fraction(float(A[i, j])) for j in range(n)] for i in range(n)]
    ipiv = []
    min_gap = float("inf")
    for k in range(n):
        mags = [abs(M[i][k]) for i in range(k, n)]
        best = max(mags)
        p = k + mags.index(best)
        if len(mags) > 1 and best != 0:
            second = sorted(mags)[-2]
            min_gap = min(min_gap, float((best - second) / best))
        ipiv.append(p)
        if M[p][k] != 0:
            M[k], M[p] = M[p], M[k]
            for i in range(k + 1, n):
                M[i][k] = M[i][k] / M[k][k]
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                M[i][j] = M[i][j] - M[i][k] * M[k][j]
    L = [[(M[i][j] if i > j else Fraction(int(i == j))) for j in range(n)] for i in range(n)]
    U = [[(M[i][j] if i <= j else Fraction(0)) for j in range(n)] for i in range(n)]
    return ipiv, L, U, min_gap


def _perm_sign(p) -> int:
    p = list(p)
    s = 1
    for i in range(len(p)):
        while p[i] != i:
            j = p[i]
            p[i], p[j] = p[j], p[i]
            s = -s
    return s


def leibniz_det(A: np.ndarray) -> Fraction:
    n = A.shape[0]
    M = [[Fraction(float(A[i, j])) for j in range(n)] for i in range(n)]
    tot = Fraction(0)
    for p in itertools.permutations(range(n)):
        term = Fraction(_perm_sign(p))
        for i in range(n):
            term *= M[i][p[i]]
            if term == 0:
                break
        tot += term
    return tot


def planted_ipiv(perm: np.ndarray) -> np.ndarray:
    """Pivot sequence for A with row perm[i] = row i of L U (|l_ij| < 1).

    At step k the reduced column is U[k,k] * L[k:, k] in the row order of L U,
    whose unique largest entry is L U's row k (l_kk = 1 > |l_ik|); that row
    currently sits at position pos[k].  Swapping positions k and pos[k] moves
    whatever L U row sat at k to pos[k].
    """
    n = len(perm)
    pos = np.array(perm, dtype=np.int64)          # pos[i]: position of L U row i
    at = np.empty(n, dtype=np.int64)              # at[r]: L U row held at position r
    at[pos] = np.arange(n)
    ipiv = np.empty(n, dtype=np.int32)
    for k in range(n):
        p = int(pos[k])
        ipiv[k] = p
        q = int(at[k])
        at[p], pos[q] = q, p
        at[k], pos[k] = k, k
    return ipiv
