"""CPU oracle for LU with partial pivoting -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The product library never loads it,
and it shares no code with the GPU path.

Contents
--------
* ``getrf`` / ``getrs``: ctypes wrappers over ``lu_oracle.c`` -- plain FP64
  Gaussian elimination with partial pivoting, one column at a time (the getf2
  form of the LAPACK getrf decomposition the paper describes in Sec. 3.4, and
  operations RL1-RL3 of LU_blk in Sec. 3.5), and the matching solve.
* ``perm_from_ipiv``, ``unpack``: turn LAPACK-style pivots / packed factors into
  a permutation vector and explicit L, U.
* ``r_factor``: scaled factorization residual ||P A - L U||_F / (||A||_F n eps).
* ``r_hpl``: HPL-style scaled solve residual
  ||A x - b||_inf / (eps (||A||_inf ||x||_inf + ||b||_inf) n).
  Both use eps = 2**-53 (unit roundoff of binary64).
* ``potrf``: ctypes wrapper over ``chol_oracle.c`` -- plain FP64 Cholesky
  A = L L^T of the lower triangle, one column at a time (the unblocked form of
  a factorization that fits the blocked skeleton of Sec. 3.1); ``r_chol``:
  scaled residual ||A - L L^T||_F / (||A||_F n eps).
* ``geqrf``: ctypes wrapper over ``qr_oracle.c`` -- plain FP64 Householder QR
  (geqr2 storage: R on and above the diagonal, reflectors below, tau);
  ``q_from`` builds Q explicitly from the reflectors.
* ``gebrd_band``: ctypes wrapper over ``band_oracle.c`` -- plain FP64
  two-sided reduction to upper band form (first stage of the SVD, the third
  workload of Sec. 6); ``band_part`` extracts the band, ``band_uv`` builds the
  orthogonal factors U, V from the stored reflectors (A = U B V^T).
* ``mlp``: FP64 forward/backward/Adam of the schedule-selector network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lu_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "chol_oracle.c"), os.path.join(_HERE, "qr_oracle.c"),
         os.path.join(_HERE, "band_oracle.c")]
_LIB = os.path.join(_HERE, "liblu_oracle.so")

EPS64 = 2.0 ** -53


def build(force: bool = False) -> str:
    """Compile lu_oracle.c with gcc (separately rounded FP ops: -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-pthread", "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_getrf.restype = ctypes.c_int
        lib.oracle_getrf.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_int]
        lib.oracle_getrs.restype = ctypes.c_int
        lib.oracle_getrs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_geqrf.restype = ctypes.c_int
        lib.oracle_geqrf.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_int]
        lib.oracle_potrf.restype = ctypes.c_int
        lib.oracle_potrf.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        lib.oracle_gebrd_band.restype = ctypes.c_int
        lib.oracle_gebrd_band.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def _as_colmajor(A: np.ndarray) -> tuple[np.ndarray, int]:
    """Return (array, lda) for a Fortran-ordered float64 view (copy if needed)."""
    if A.dtype != np.float64:
        raise TypeError("oracle works in float64")
    if A.ndim != 2:
        raise ValueError("matrix expected")
    if A.strides[0] != 8:
        A = np.asfortranarray(A)
    lda = A.strides[1] // 8 if A.shape[1] > 1 else max(1, A.shape[0])
    return A, lda


def getrf(A: np.ndarray, nthreads: int = 1, copy: bool = True):
    """Factor the square matrix A: returns (LU, ipiv (int32, 0-based), info)."""
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("square matrix expected")
    LU = np.array(A, dtype=np.float64, order="F", copy=True) if copy else A
    LU, lda = _as_colmajor(LU)
    ipiv = np.zeros(max(n, 1), dtype=np.int32)
    info = _load().oracle_getrf(n, LU.ctypes.data, max(lda, 1), ipiv.ctypes.data, int(nthreads))
    if info < 0:
        raise ValueError("oracle_getrf: illegal argument %d" % -info)
    return LU, ipiv[:n], info


def getrs(LU: np.ndarray, ipiv: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve A X = B from getrf's output; returns X (B is not modified)."""
    n = LU.shape[0]
    LU, lda = _as_colmajor(LU)
    vec = B.ndim == 1
    X = np.array(B.reshape(n, -1), dtype=np.float64, order="F", copy=True)
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    r = _load().oracle_getrs(n, X.shape[1], LU.ctypes.data, max(lda, 1), ipiv.ctypes.data,
                             X.ctypes.data, max(n, 1))
    if r != 0:
        raise ValueError("oracle_getrs: illegal argument %d" % -r)
    return X[:, 0] if vec else X


def potrf(A: np.ndarray, nthreads: int = 1):
    """Cholesky of the lower triangle of the SPD matrix A: returns (F, info)
    where tril(F) = L and the strictly upper triangle of F is A's, untouched."""
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("square matrix expected")
    F = np.array(A, dtype=np.float64, order="F", copy=True)
    F, lda = _as_colmajor(F)
    info = _load().oracle_potrf(n, F.ctypes.data, max(lda, 1), int(nthreads))
    if info < 0:
        raise ValueError("oracle_potrf: illegal argument %d" % -info)
    return F, info


def geqrf(A: np.ndarray, nthreads: int = 1):
    """Householder QR of the m x n (m >= n) matrix A: returns (F, tau)."""
    m, n = A.shape
    F = np.array(A, dtype=np.float64, order="F", copy=True)
    F, lda = _as_colmajor(F)
    tau = np.zeros(max(n, 1), dtype=np.float64)
    rc = _load().oracle_geqrf(m, n, F.ctypes.data, max(lda, 1), tau.ctypes.data, int(nthreads))
    if rc < 0:
        raise ValueError("oracle_geqrf: illegal argument %d" % -rc)
    return F, tau[:n]


def q_from(F: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Q = H_0 H_1 ... H_{n-1}, H_j = I - tau_j v_j v_j^T (m x m), from geqrf's output."""
    m, n = F.shape
    Q = np.eye(m)
    for j in range(n - 1, -1, -1):
        v = np.zeros(m)
        v[j] = 1.0
        v[j + 1:] = F[j + 1:, j]
        Q = Q - tau[j] * np.outer(v, v @ Q)
    return Q


def gebrd_band(A: np.ndarray, w: int):
    """Two-sided reduction of the square matrix A to upper band form with
    bandwidth w: returns (F, tauq, taup) in the storage band_oracle.c
    describes."""
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("square matrix expected")
    F = np.array(A, dtype=np.float64, order="F", copy=True)
    F, lda = _as_colmajor(F)
    tauq = np.zeros(max(n, 1), dtype=np.float64)
    taup = np.zeros(max(n, 1), dtype=np.float64)
    rc = _load().oracle_gebrd_band(n, int(w), F.ctypes.data, max(lda, 1), tauq.ctypes.data, taup.ctypes.data)
    if rc < 0:
        raise ValueError("oracle_gebrd_band: illegal argument %d" % -rc)
    return F, tauq[:n], taup[:n]


def band_part(F: np.ndarray, w: int) -> np.ndarray:
    """The band B of a reduced matrix: entries (i, j) with 0 <= j - i <= w."""
    n = F.shape[0]
    i, j = np.indices((n, n))
    return np.where((j - i >= 0) & (j - i <= w), F, 0.0)


def band_uv(F: np.ndarray, tauq: np.ndarray, taup: np.ndarray, w: int):
    """U = H_0 H_1 ... (column reflectors) and V = G_0 G_1 ... (row
    reflectors) of a band reduction, so that A = U B V^T."""
    n = F.shape[0]
    U = np.eye(n)
    for j in range(n - 1, -1, -1):
        v = np.zeros(n)
        v[j] = 1.0
        v[j + 1:] = F[j + 1:, j]
        U = U - tauq[j] * np.outer(v, v @ U)
    V = np.eye(n)
    for r in range(n - 1, -1, -1):
        c = (r // w) * w + w + (r % w)
        if c >= n:
            continue
        v = np.zeros(n)
        v[c] = 1.0
        v[c + 1:] = F[r, c + 1:]
        V = V - taup[r] * np.outer(v, v @ V)
    return U, V


def r_chol(A: np.ndarray, F: np.ndarray, matmul=None) -> float:
    """Scaled Cholesky residual ||A - L L^T||_F / (||A||_F n eps), L = tril(F)."""
    n = A.shape[0]
    if n == 0:
        return 0.0
    L = np.tril(F)
    LLt = (matmul or np.matmul)(L, L.T)
    return float(np.linalg.norm(A - LLt) / (np.linalg.norm(A) * n * EPS64))


def perm_from_ipiv(ipiv: np.ndarray) -> np.ndarray:
    """Row permutation p with (P A)[i, :] = A[p[i], :], from sequential interchanges."""
    n = len(ipiv)
    p = np.arange(n)
    for k in range(n):
        j = int(ipiv[k])
        if j != k:
            p[k], p[j] = p[j], p[k]
    return p


def unpack(LU: np.ndarray):
    """Explicit unit-lower L and upper U from the packed factor."""
    L = np.tril(LU, -1)
    np.fill_diagonal(L, 1.0)
    return L, np.triu(LU)


def r_factor(A: np.ndarray, LU: np.ndarray, ipiv: np.ndarray, matmul=None) -> float:
    """||P A - L U||_F / (||A||_F * n * eps) in FP64.

    ``matmul`` (optional) computes L @ U; the default is numpy's.
    """
    n = A.shape[0]
    if n == 0:
        return 0.0
    L, U = unpack(np.asarray(LU))
    prod = (matmul or np.matmul)(L, U)
    PA = np.asarray(A)[perm_from_ipiv(ipiv), :]
    na = np.linalg.norm(A, "fro")
    if na == 0.0:
        return 0.0 if np.linalg.norm(PA - prod) == 0.0 else float("inf")
    return float(np.linalg.norm(PA - prod, "fro") / (na * n * EPS64))


def r_hpl(A: np.ndarray, x: np.ndarray, b: np.ndarray) -> float:
    """HPL 2.x acceptance residual ||A x - b||_inf / (eps (||A||_inf ||x||_inf + ||b||_inf) n)."""
    n = A.shape[0]
    r = A @ x - b
    na = np.abs(A).sum(axis=1).max()
    denom = EPS64 * (na * np.abs(x).max() + np.abs(b).max()) * n
    return float(np.abs(r).max() / denom)


def solve(A: np.ndarray, b: np.ndarray, nthreads: int = 1) -> np.ndarray:
    """FP64 oracle solution x_o of A x = b (factor + solve)."""
    LU, ipiv, info = getrf(A, nthreads=nthreads)
    if info != 0:
        raise np.linalg.LinAlgError("singular matrix (info=%d)" % info)
    return getrs(LU, ipiv, b)
