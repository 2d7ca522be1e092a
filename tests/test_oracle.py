"""Pins for the CPU oracle (no GPU).  Each pin is independent of the oracle's
own code: exact rational elimination, Leibniz determinants, a hand-worked
example, planted factors, LAPACK's dgetrf, backward-error bounds and special
cases whose answer is known in closed form.  ``test_mutants_are_caught``
plants typical mistakes into copies of the oracle source and checks that the
pins reject every one of them.
"""
import os
import re
import shutil
import subprocess
import ctypes
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg.lapack as lapack

import oracle
import synth
from tests import pins

HERE = os.path.dirname(os.path.abspath(__file__))


def _frac_matrix(rows):
    return [[Fraction(x) for x in r.split()] for r in rows]


def _read_golden(name):
    blocks, cur = {}, None
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if re.fullmatch(r"[A-Za-z]+", line):
                cur = line
                blocks[cur] = []
            else:
                blocks[cur].append(line)
    return blocks


def test_hand_worked_3x3():
    g = _read_golden("lu3x3_hand.txt")
    A = np.array([[float(Fraction(x)) for x in r.split()] for r in g["A"]], order="F")
    LU, ipiv, info = oracle.getrf(A)
    assert info == 0
    assert list(ipiv) == [int(x) for x in g["ipiv"][0].split()]
    L, U = oracle.unpack(LU)
    Lx, Ux = _frac_matrix(g["L"]), _frac_matrix(g["U"])
    for i in range(3):
        for j in range(3):
            assert L[i, j] == pytest.approx(float(Lx[i][j]), abs=1e-15)
            assert U[i, j] == pytest.approx(float(Ux[i][j]), abs=1e-14)
    det = np.prod(np.diag(U)) * (-1) ** int(np.sum(ipiv != np.arange(3)))
    assert det == pytest.approx(float(Fraction(g["det"][0])), rel=1e-14)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_exact(n, seed):
    A = synth.uniform(n, seed=seed)
    LU, ipiv, info = oracle.getrf(A)
    eipiv, eL, eU, gap = pins.exact_gepp(A)
    assert info == 0
    if gap > 1e-10:
        assert list(ipiv) == eipiv
        L, U = oracle.unpack(LU)
        for i in range(n):
            for j in range(n):
                assert abs(L[i, j] - float(eL[i][j])) <= 1e-12
                assert abs(U[i, j] - float(eU[i][j])) <= 1e-12 * max(1.0, abs(float(eU[i][j])))
    if n <= 7:
        det = pins.leibniz_det(A)
        sign = (-1) ** int(np.sum(ipiv != np.arange(n)))
        got = sign * np.prod(np.diag(LU))
        assert got == pytest.approx(float(det), rel=1e-12, abs=1e-14)


def test_n1_and_2x2_by_hand():
    LU, ipiv, info = oracle.getrf(np.array([[-3.5]], order="F"))
    assert info == 0 and list(ipiv) == [0] and LU[0, 0] == -3.5
    # |a21| > |a11| -> swap
    LU, ipiv, info = oracle.getrf(np.array([[1.0, 2.0], [-4.0, 8.0]], order="F"))
    assert list(ipiv) == [1, 1]
    assert LU[0, 0] == -4.0 and LU[0, 1] == 8.0
    assert LU[1, 0] == -0.25 and LU[1, 1] == 2.0 - (-0.25) * 8.0
    # |a21| < |a11| -> no swap
    LU, ipiv, info = oracle.getrf(np.array([[4.0, 1.0], [2.0, 3.0]], order="F"))
    assert list(ipiv) == [0, 1] and LU[1, 0] == 0.5 and LU[1, 1] == 2.5


def test_identity_and_permutation():
    n = 9
    LU, ipiv, info = oracle.getrf(np.eye(n, order="F"))
    assert info == 0 and list(ipiv) == list(range(n))
    assert np.array_equal(LU, np.eye(n))
    perm = synth.rng(5, 2).permutation(n)
    A = np.asfortranarray(np.eye(n)[perm, :])          # row i of A is e_{perm[i]}
    LU, ipiv, info = oracle.getrf(A)
    assert np.array_equal(LU, np.eye(n))               # L = U = I bitwise
    P = oracle.perm_from_ipiv(ipiv)
    assert np.array_equal(A[P, :], np.eye(n))


def test_upper_triangular_is_its_own_u():
    n = 12
    A = np.triu(synth.uniform(n, seed=4)) + 3.0 * np.eye(n)
    A = np.asfortranarray(A)
    LU, ipiv, info = oracle.getrf(A)
    assert list(ipiv) == list(range(n))
    assert np.array_equal(LU, A)


def test_zero_column_and_zero_matrix():
    n = 10
    A = synth.uniform(n, seed=7)
    A[:, 4] = 0.0
    _, ipiv, info = oracle.getrf(A)
    assert info == 5
    _, ipiv, info = oracle.getrf(np.zeros((n, n), order="F"))
    assert info == 1 and list(ipiv) == list(range(n))


def test_ties_take_smallest_index():
    A = np.asfortranarray(np.array([[1.0, 5.0, 0.0],
                                    [-1.0, 2.0, 1.0],
                                    [1.0, -3.0, 4.0]]))
    _, ipiv, _ = oracle.getrf(A)
    assert ipiv[0] == 0
    A2 = np.asfortranarray(np.array([[0.5, 0.0], [-2.0, 1.0]]))
    B = np.asfortranarray(np.array([[0.5, 1.0, 0.0], [2.0, 0.0, 1.0], [-2.0, 3.0, 2.0]]))
    _, ipiv, _ = oracle.getrf(B)
    assert ipiv[0] == 1                                 # |2| == |-2|: first index wins
    _, ipiv, _ = oracle.getrf(A2)
    assert ipiv[0] == 1


@pytest.mark.parametrize("n", [64, 256, 512])
def test_planted_factors_recovered(n):
    A, L, U, perm = synth.planted(n, seed=3)
    LU, ipiv, info = oracle.getrf(A, nthreads=4)
    assert info == 0
    assert np.array_equal(ipiv, pins.planted_ipiv(perm))
    Lh, Uh = oracle.unpack(LU)
    assert np.abs(Lh - L).max() <= 1e-12
    assert np.abs(Uh - U).max() <= 1e-12 * np.abs(U).max()


@pytest.mark.parametrize("n", [200, 512])
def test_matches_lapack_dgetrf(n):
    A = synth.uniform(n, seed=11)
    LU, ipiv, info = oracle.getrf(A, nthreads=4)
    lu_ref, piv_ref, info_ref = lapack.dgetrf(np.array(A))
    assert info == info_ref == 0
    assert np.array_equal(ipiv, piv_ref)               # scipy returns 0-based pivots
    assert np.abs(LU - lu_ref).max() <= 1e-12 * np.abs(lu_ref).max()


@pytest.mark.parametrize("n,seed", [(100, 1), (333, 2), (512, 3)])
def test_backward_error_bound(n, seed):
    A = synth.uniform(n, seed=seed)
    LU, ipiv, info = oracle.getrf(A, nthreads=3)
    assert oracle.r_factor(A, LU, ipiv) <= 16.0


def test_thread_count_bitwise():
    A = synth.uniform(300, seed=9)
    a1 = oracle.getrf(A, nthreads=1)
    a5 = oracle.getrf(A, nthreads=5)
    assert np.array_equal(a1[0], a5[0]) and np.array_equal(a1[1], a5[1])


def test_lda_padding_untouched():
    A = synth.uniform(50, seed=2, lda=57)
    LU, ipiv, info = oracle.getrf(A, copy=False)
    base = A.base if A.base is not None else A
    assert np.isnan(np.asarray(base)[50:, :]).all()
    assert oracle.r_factor(synth.uniform(50, seed=2), LU, ipiv) <= 16.0


@pytest.mark.parametrize("n", [1, 17, 256])
def test_solve_residual(n):
    A = synth.uniform(n, seed=5)
    b = synth.rhs(n, seed=5)[:, 0]
    x = oracle.solve(A, b)
    assert oracle.r_hpl(A, x, b) <= 16.0
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10)


def test_dominant_makes_no_swaps():
    A = synth.dominant(128, seed=1)
    _, ipiv, _ = oracle.getrf(A)
    assert np.array_equal(ipiv, np.arange(128))


# ---------------------------------------------------------------- mutants
MUTANTS = {
    "no_abs_in_pivot": ("double v = fabs(AT(A, lda, i, k));", "double v = AT(A, lda, i, k);"),
    "last_index_on_ties": ("if (v > best)", "if (v >= best)"),
    "no_swap_of_left_columns": ("split(0, n, w->nthreads", "split(k, n, w->nthreads"),
    "update_sign": ("col[i] = col[i] - prod;", "col[i] = col[i] + prod;"),
    "scale_by_multiply": ("AT(A, lda, i, k) / piv;", "AT(A, lda, i, k) * piv;"),
    "update_wrong_row_start": ("for (int i = k + 1; i < n; ++i) {\n                    double prod",
                               "for (int i = k; i < n; ++i) {\n                    double prod"),
    "solve_without_swaps": ("if (p != k) { double t = b[k];", "if (0) { double t = b[k];"),
}


def _pins_pass(lib) -> bool:
    def getrf(A):
        LU = np.array(A, order="F", copy=True)
        ip = np.zeros(LU.shape[0], dtype=np.int32)
        info = lib.oracle_getrf(LU.shape[0], LU.ctypes.data, LU.shape[0], ip.ctypes.data, 2)
        return LU, ip, info

    ok = True
    for n, seed in [(5, 1), (6, 2)]:                       # exact brute force
        A = synth.uniform(n, seed=seed)
        LU, ip, _ = getrf(A)
        e_ip, eL, eU, _ = pins.exact_gepp(A)
        ok &= list(ip) == e_ip
        ok &= all(abs(LU[i, j] - float((eL if i > j else eU)[i][j])) < 1e-12
                  for i in range(n) for j in range(n))
    A = np.asfortranarray(np.array([[0.5, 1.0, 0.0], [2.0, 0.0, 1.0], [-2.0, 3.0, 2.0]]))
    ok &= getrf(A)[1][0] == 1                               # tie rule
    A, L, U, perm = synth.planted(64, seed=3)               # planted factors
    LU, ip, _ = getrf(A)
    ok &= np.array_equal(ip, pins.planted_ipiv(perm))
    A = synth.uniform(64, seed=4)                           # backward error + solve
    LU, ip, _ = getrf(A)
    ok &= oracle.r_factor(A, LU, ip) <= 16.0
    b = synth.rhs(64, seed=4)[:, 0].copy()
    x = b.copy()
    lib.oracle_getrs(64, 1, LU.ctypes.data, 64, ip.ctypes.data, x.ctypes.data, 64)
    ok &= oracle.r_hpl(A, x, b) <= 16.0
    return bool(ok)


def _build_variant(tmp_path, name, src):
    cpath = tmp_path / (name + ".c")
    cpath.write_text(src)
    so = tmp_path / (name + ".so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                           "-o", str(so), str(cpath), "-lm"])
    lib = ctypes.CDLL(str(so))
    lib.oracle_getrf.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
    lib.oracle_getrs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    return lib


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc needed")
def test_mutants_are_caught(tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "lu_oracle.c")).read()
    assert _pins_pass(_build_variant(tmp_path, "unmodified", src))
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, name
        lib = _build_variant(tmp_path, name, src.replace(old, new))
        assert not _pins_pass(lib), "pins did not catch mutant " + name
