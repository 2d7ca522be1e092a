"""Pins of the CPU band-reduction oracle (oracle/band_oracle.c) against facts
that do not come from the oracle itself: a 3 x 3 worked by hand, the singular
values of A (LAPACK gesdd through numpy), the defining relation A = U B V^T
with U, V orthogonal and B banded (U, V built here from the stored reflectors),
the special cases that reduce to Householder QR (w >= n, and the first column
panel), and a mutation test of plausible mistakes in the C source."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth


def test_hand_3x3_w1():
    # H_0 from (3, 4, 0): beta -5, tau 1.6, v = (1, 0.5, 0); it maps column 1
    # (-5, 0, 1) to (3, 4, 1) and column 2 (0, -5, 2) to (4, -3, 2).  G_0 from
    # row 0's (3, 4): beta -5, tau 1.6, v = (1, 0.5); rows 1, 2 become (0, -5),
    # (-2.2, 0.4).  H_1 from (0, -2.2): beta -2.2, tau 1, v = (1, -1); column 2
    # (-5, 0.4) -> (0.4, -5).  The remaining reflectors have length 1 (tau 0).
    A = np.array([[3.0, -5.0, 0.0], [4.0, 0.0, -5.0], [0.0, 1.0, 2.0]])
    F, tauq, taup = oracle.gebrd_band(A, 1)
    want = np.array([[-5.0, -5.0, 0.5], [0.5, -2.2, 0.4], [0.0, -1.0, -5.0]])
    assert np.abs(F - want).max() <= 8 * 2.0 ** -52 * 5
    assert np.abs(tauq - [1.6, 1.0, 0.0]).max() <= 4e-16
    assert np.abs(taup - [1.6, 0.0, 0.0]).max() <= 4e-16


@pytest.mark.parametrize("n,w", [(30, 1), (64, 8), (100, 16), (97, 12), (130, 32), (45, 44)])
def test_singular_values_preserved(n, w):
    A = synth.uniform(n, seed=n * 7 + w)
    F, _, _ = oracle.gebrd_band(A, w)
    sa = np.linalg.svd(A, compute_uv=False)
    sb = np.linalg.svd(oracle.band_part(F, w), compute_uv=False)
    assert np.abs(sa - sb).max() <= 1e-13 * sa[0]


@pytest.mark.parametrize("n,w", [(40, 4), (57, 8), (33, 40)])
def test_a_equals_u_b_vt(n, w):
    A = synth.uniform(n, seed=n + w)
    F, tauq, taup = oracle.gebrd_band(A, w)
    B = oracle.band_part(F, w)
    U, V = oracle.band_uv(F, tauq, taup, w)
    assert np.abs(U.T @ U - np.eye(n)).max() <= 1e-14 * n
    assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-14 * n
    assert np.abs(U @ B @ V.T - A).max() <= 1e-14 * n
    # everything outside the band is annihilated
    assert np.abs(U.T @ A @ V - B).max() <= 1e-14 * n
    # rows without a reflector: the last band of rows and rows whose segment is empty
    for r in range(n):
        c = (r // w) * w + w + (r % w)
        if c >= n:
            assert taup[r] == 0.0


@pytest.mark.parametrize("n,w", [(20, 20), (20, 64), (37, 37)])
def test_w_at_least_n_is_householder_qr(n, w):
    A = synth.uniform(n, seed=3 * n)
    F, tauq, taup = oracle.gebrd_band(A, w)
    Fq, tq = oracle.geqrf(A)
    assert np.array_equal(F, Fq) and np.array_equal(tauq, tq)
    assert not taup.any()


def test_first_column_panel_is_householder_qr():
    n, w = 60, 12
    A = synth.uniform(n, seed=77)
    F, tauq, _ = oracle.gebrd_band(A, w)
    Fq, tq = oracle.geqrf(np.asfortranarray(A[:, :w]))
    assert np.array_equal(F[:, :w], Fq) and np.array_equal(tauq[:w], tq)


def test_zero_and_identity():
    F, tauq, taup = oracle.gebrd_band(np.zeros((6, 6)), 2)
    assert not F.any() and not tauq.any() and not taup.any()
    F, tauq, taup = oracle.gebrd_band(np.eye(7), 3)
    assert np.array_equal(F, np.eye(7)) and not tauq.any() and not taup.any()


# ---------------------------------------------------------------- mutation test
MUTANTS = {
    "sign_of_beta": ("const double beta = alpha >= 0.0 ? -nrm : nrm;", "const double beta = alpha >= 0.0 ? nrm : -nrm;"),
    "tau_formula": ("const double tau = (beta - alpha) / beta;", "const double tau = (beta - alpha) / alpha;"),
    "left_update_sign": ("        const double t = -tau * d;", "        const double t = tau * d;"),
    "right_dot_without_first": ("for (int q = r + 1; q < n; ++q) d[q] = AT(A, lda, q, c);",
                                "for (int q = r + 1; q < n; ++q) d[q] = 0.0;"),
    "right_first_column_skipped": ("for (int q = r + 1; q < n; ++q) AT(A, lda, q, c) = AT(A, lda, q, c) + d[q];",
                                   "for (int q = r + 1; q < n; ++q) AT(A, lda, q, c) = AT(A, lda, q, c);"),
    "right_rows_of_panel_skipped": ("if (taup[r] != 0.0) band_right(A, lda, n, r, c, taup[r], d);",
                                    "if (taup[r] != 0.0) band_right(A, lda, n, k + kw - 1 > r ? k + kw - 1 : r, c, taup[r], d);"),
    "row_panel_offset": ("const int r = k + i, c = k + w + i;", "const int r = k + i, c = k + w + i - 1;"),
    "no_right_side": ("if (taup[r] != 0.0) band_right(", "if (0) band_right("),
}


def _pins_pass(lib):
    def run(A, w):
        F = np.array(A, dtype=np.float64, order="F", copy=True)
        n = F.shape[0]
        tq, tp = np.zeros(n), np.zeros(n)
        lib.oracle_gebrd_band(n, w, F.ctypes.data, n, tq.ctypes.data, tp.ctypes.data)
        return F, tq, tp
    ok = True
    F, tq, tp = run(np.array([[3.0, -5.0, 0.0], [4.0, 0.0, -5.0], [0.0, 1.0, 2.0]]), 1)
    ok &= np.abs(F - np.array([[-5.0, -5.0, 0.5], [0.5, -2.2, 0.4], [0.0, -1.0, -5.0]])).max() <= 4e-15
    ok &= np.abs(tq - [1.6, 1.0, 0.0]).max() <= 4e-16 and np.abs(tp - [1.6, 0.0, 0.0]).max() <= 4e-16
    for n, w in [(30, 4), (25, 3)]:
        A = synth.uniform(n, seed=n)
        F, tq, tp = run(A, w)
        B = oracle.band_part(F, w)
        sa = np.linalg.svd(A, compute_uv=False)
        ok &= bool(np.abs(sa - np.linalg.svd(B, compute_uv=False)).max() <= 1e-13 * sa[0])
        U, V = oracle.band_uv(F, tq, tp, w)
        ok &= bool(np.abs(U @ B @ V.T - A).max() <= 1e-13)
    return bool(ok)


def _build_variant(tmp_path, name, src):
    cpath = tmp_path / (name + ".c")
    cpath.write_text(src)
    so = tmp_path / (name + ".so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(so), str(cpath),
                           "-lm"])
    lib = ctypes.CDLL(str(so))
    lib.oracle_gebrd_band.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_void_p]
    lib.oracle_gebrd_band.restype = ctypes.c_int
    return lib


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc needed")
def test_mutants_are_caught(tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "band_oracle.c")).read()
    assert _pins_pass(_build_variant(tmp_path, "unmodified", src))
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, name
        lib = _build_variant(tmp_path, name, src.replace(old, new))
        assert not _pins_pass(lib), "pins did not catch mutant " + name
