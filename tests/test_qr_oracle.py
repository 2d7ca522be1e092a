"""Pins of the CPU Householder QR oracle (oracle/qr_oracle.c) against facts
that do not come from the oracle itself: a 2 x 2 worked by hand, LAPACK dgeqrf
(the same reflector convention), the defining properties Q R = A and Q^T Q = I
with Q built from the reflectors, closed-form special cases, determinism over
thread counts, and a mutation test of plausible mistakes in the C source."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.linalg.lapack as lapack

import oracle
import synth


def test_hand_2x2():
    # column 0: alpha 3, |x| 4 -> beta -5, tau (-5-3)/-5 = 1.6, v1 = 4/(3+5) = 0.5
    # column 1: w = 1 + 0.5*2 = 2 -> R01 = 1 - 1.6*2 = -2.2, A11 = 2 - 0.5*1.6*2 = 0.4
    F, tau = oracle.geqrf(np.array([[3.0, 1.0], [4.0, 2.0]], order="F"))
    want_F = np.array([[-5.0, -2.2], [0.5, 0.4]])
    assert np.abs(F - want_F).max() <= 4e-16 * 5
    assert abs(tau[0] - 1.6) <= 4e-16 and tau[1] == 0.0


@pytest.mark.parametrize("m,n", [(50, 50), (300, 300), (257, 100)])
def test_matches_lapack_dgeqrf(m, n):
    A = synth.uniform(m, seed=m + n)[:, :n].copy(order="F")
    F, tau = oracle.geqrf(A, nthreads=4)
    qr, ltau, _, info = lapack.dgeqrf(A)
    assert info == 0
    assert np.abs(F - qr).max() <= 1e-13 * max(1.0, np.abs(qr).max())
    assert np.abs(tau - ltau[:n]).max() <= 1e-13


@pytest.mark.parametrize("m,n", [(40, 40), (64, 17)])
def test_q_times_r_is_a(m, n):
    A = synth.uniform(m, seed=7)[:, :n].copy(order="F")
    F, tau = oracle.geqrf(A)
    Q = oracle.q_from(F, tau)
    R = np.triu(F)[:n, :]
    assert np.abs(Q[:, :n] @ R - A).max() <= 1e-13 * n
    assert np.abs(Q.T @ Q - np.eye(m)).max() <= 1e-13 * m


def test_special_cases():
    F, tau = oracle.geqrf(np.eye(6, order="F"))
    assert np.array_equal(tau, np.zeros(6)) and np.array_equal(F, np.eye(6))
    A = synth.uniform(8, seed=3)
    A[1:, 0] = 0.0                       # column 0 already upper: H_0 = I
    F, tau = oracle.geqrf(A)
    assert tau[0] == 0.0 and F[0, 0] == A[0, 0]
    A = np.zeros((5, 5), order="F")
    F, tau = oracle.geqrf(A)
    assert np.array_equal(F, A) and np.array_equal(tau, np.zeros(5))


def test_thread_count_bitwise():
    A = synth.uniform(200, seed=9)
    F1, t1 = oracle.geqrf(A, nthreads=1)
    F8, t8 = oracle.geqrf(A, nthreads=8)
    assert np.array_equal(F1, F8) and np.array_equal(t1, t8)


# ---------------------------------------------------------------- mutation test
MUTANTS = {
    "sign_of_beta": ("const double beta = alpha >= 0.0 ? -nrm : nrm;", "const double beta = alpha >= 0.0 ? nrm : -nrm;"),
    "norm_without_alpha": ("double nrm = sqrt(a2 + s);", "double nrm = sqrt(s);"),
    "tau_formula": ("w->tau[j] = (beta - alpha) / beta;", "w->tau[j] = (beta - alpha) / alpha;"),
    "no_scaling": ("for (int i = j + 1; i < m; ++i) AT(A, lda, i, j) = AT(A, lda, i, j) * scal;",
                   "for (int i = j + 1; i < m; ++i) AT(A, lda, i, j) = AT(A, lda, i, j);"),
    "w_without_diag": ("double wc = AT(A, lda, j, c);", "double wc = 0.0;"),
    "update_sign": ("const double t = -tau * wc;", "const double t = tau * wc;"),
    "diag_row_not_updated": ("AT(A, lda, j, c) = AT(A, lda, j, c) + t;", "AT(A, lda, j, c) = AT(A, lda, j, c);"),
}


def _pins_pass(lib):
    def run(A, nt=1):
        F = np.array(A, dtype=np.float64, order="F", copy=True)
        tau = np.zeros(F.shape[1])
        lib.oracle_geqrf(F.shape[0], F.shape[1], F.ctypes.data, F.shape[0], tau.ctypes.data, nt)
        return F, tau
    ok = True
    F, tau = run(np.array([[3.0, 1.0], [4.0, 2.0]]))
    ok &= np.abs(F - np.array([[-5.0, -2.2], [0.5, 0.4]])).max() <= 2e-15 and abs(tau[0] - 1.6) <= 4e-16
    A = synth.uniform(30, seed=5)
    F, tau = run(A, 3)
    qr, ltau, _, _ = lapack.dgeqrf(A)
    ok &= np.abs(F - qr).max() <= 1e-13 * np.abs(qr).max() and np.abs(tau - ltau).max() <= 1e-13
    return bool(ok)


def _build_variant(tmp_path, name, src):
    cpath = tmp_path / (name + ".c")
    cpath.write_text(src)
    so = tmp_path / (name + ".so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                           "-o", str(so), str(cpath), "-lm"])
    lib = ctypes.CDLL(str(so))
    lib.oracle_geqrf.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                 ctypes.c_int]
    lib.oracle_geqrf.restype = ctypes.c_int
    return lib


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc needed")
def test_mutants_are_caught(tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "qr_oracle.c")).read()
    assert _pins_pass(_build_variant(tmp_path, "unmodified", src))
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, name
        lib = _build_variant(tmp_path, name, src.replace(old, new))
        assert not _pins_pass(lib), "pins did not catch mutant " + name
