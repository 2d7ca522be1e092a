"""Pins of the CPU Cholesky oracle (oracle/chol_oracle.c) against facts that do
not come from the oracle itself: a factorization worked by hand, integer
factors recovered exactly (every intermediate value is an integer, every
square root a perfect square), LAPACK's potrf through numpy, the LAPACK
definition of a non-positive pivot, and determinism over thread counts.  A
mutation test checks that plausible mistakes in the C source fail the pins."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth


def test_hand_2x2():
    # [[4, 2], [2, 5]] = [[2, 0], [1, 2]] [[2, 1], [0, 2]]
    A = np.array([[4.0, 2.0], [2.0, 5.0]], order="F")
    F, info = oracle.potrf(A)
    assert info == 0
    assert np.array_equal(np.tril(F), np.array([[2.0, 0.0], [1.0, 2.0]]))
    assert F[0, 1] == 2.0                      # strictly upper triangle untouched


def _integer_factor(n, seed):
    r = np.random.default_rng(seed)
    L = np.tril(r.integers(-3, 4, size=(n, n)), -1) + np.diag(r.integers(1, 5, size=n))
    A = (L @ L.T).astype(np.float64)            # exact: small integers
    return L.astype(np.float64), np.asfortranarray(A)


@pytest.mark.parametrize("n,seed", [(1, 0), (3, 1), (17, 2), (60, 3)])
def test_integer_factors_recovered_exactly(n, seed):
    L, A = _integer_factor(n, seed)
    F, info = oracle.potrf(A, nthreads=3)
    assert info == 0
    assert np.array_equal(np.tril(F), L)
    assert np.array_equal(np.triu(F, 1), np.triu(A, 1))


def test_identity_and_diagonal():
    F, info = oracle.potrf(np.eye(7, order="F"))
    assert info == 0 and np.array_equal(np.tril(F), np.eye(7))
    d = np.array([4.0, 2.0, 9.0, 0.25, 3.0])
    F, info = oracle.potrf(np.diag(d).copy(order="F"))
    assert info == 0 and np.array_equal(np.diag(F), np.sqrt(d))


@pytest.mark.parametrize("A,want", [
    (np.diag([1.0, -1.0, 1.0]), 2),
    (np.zeros((3, 3)), 1),
    (np.array([[1.0, 2.0], [2.0, 1.0]]), 2),     # indefinite: 1 - 2*2 < 0 at step 2
    (np.array([[1.0, 1.0], [1.0, 1.0]]), 2),     # singular: the second pivot is exactly 0
    (np.array([[np.nan, 0.0], [0.0, 1.0]]), 1),
])
def test_not_positive_definite_info(A, want):
    F, info = oracle.potrf(np.asfortranarray(A))
    assert info == want


@pytest.mark.parametrize("n", [50, 300])
def test_matches_lapack_potrf(n):
    A = synth.spd(n, seed=n)
    F, info = oracle.potrf(A, nthreads=4)
    assert info == 0
    Lref = np.linalg.cholesky(A)
    assert np.abs(np.tril(F) - Lref).max() <= 1e-13 * np.abs(Lref).max()
    assert oracle.r_chol(A, F) <= 1.0


def test_thread_count_bitwise():
    A = synth.spd(257, seed=9)
    F1, _ = oracle.potrf(A, nthreads=1)
    F8, _ = oracle.potrf(A, nthreads=8)
    assert np.array_equal(F1, F8)


def test_spd_generator():
    A = synth.spd(64, seed=2)
    assert np.array_equal(A, A.T)
    d = np.diag(A)
    off = np.abs(A).sum(axis=1) - np.abs(d)
    assert (d > off).all()                        # strictly diagonally dominant, positive diagonal


# ---------------------------------------------------------------- mutation test
MUTANTS = {
    "no_update": ("col[i] = col[i] - prod;", "col[i] = col[i];"),
    "update_from_diag_plus_one": ("for (int i = j; i < n; ++i) {", "for (int i = j + 1; i < n; ++i) {"),
    "no_sqrt": ("const double r = sqrt(d);", "const double r = d;"),
    "upper_operand": ("const double ljk = AT(A, lda, j, k);", "const double ljk = AT(A, lda, k, j);"),
    "accept_zero_pivot": ("if (!(d > 0.0)) {", "if (!(d >= 0.0)) {"),
    "scale_diag_too": ("for (int i = k + 1; i < n; ++i) AT(A, lda, i, k) = AT(A, lda, i, k) / r;",
                       "for (int i = k; i < n; ++i) AT(A, lda, i, k) = AT(A, lda, i, k) / r;"),
}


def _pins_pass(lib):
    def run(A, nt=1):
        F = np.array(A, dtype=np.float64, order="F", copy=True)
        info = lib.oracle_potrf(F.shape[0], F.ctypes.data, max(1, F.shape[0]), nt)
        return F, info
    ok = True
    F, info = run(np.array([[4.0, 2.0], [2.0, 5.0]]))
    ok &= info == 0 and np.array_equal(np.tril(F), np.array([[2.0, 0.0], [1.0, 2.0]]))
    L, A = _integer_factor(17, 2)
    F, info = run(A, 3)
    ok &= info == 0 and np.array_equal(np.tril(F), L) and np.array_equal(np.triu(F, 1), np.triu(A, 1))
    F, info = run(np.array([[1.0, 1.0], [1.0, 1.0]]))
    ok &= info == 2
    return bool(ok)


def _build_variant(tmp_path, name, src):
    cpath = tmp_path / (name + ".c")
    cpath.write_text(src)
    so = tmp_path / (name + ".so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                           "-o", str(so), str(cpath), "-lm"])
    lib = ctypes.CDLL(str(so))
    lib.oracle_potrf.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.oracle_potrf.restype = ctypes.c_int
    return lib


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc needed")
def test_mutants_are_caught(tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "chol_oracle.c")).read()
    assert _pins_pass(_build_variant(tmp_path, "unmodified", src))
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, name
        lib = _build_variant(tmp_path, name, src.replace(old, new))
        assert not _pins_pass(lib), "pins did not catch mutant " + name
