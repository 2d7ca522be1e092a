"""Pins of the scaled residuals that every acceptance test at large n rests on
(no GPU).  Each expected value is worked out by hand from the definition --
R_f = ||P A - L U||_F / (||A||_F n eps), R_hpl = ||A x - b||_inf /
(eps (||A||_inf ||x||_inf + ||b||_inf) n), R_chol = ||A - L L^T||_F /
(||A||_F n eps), eps = 2**-53 -- on 2 x 2 examples whose perturbations are
powers of two, so the floating-point evaluation is exact (or the exact value is
computed with fractions).  The examples separate the plausible slips: eps =
2**-52 halves a value, a dropped n doubles it, another norm (max, 1-norm,
2-norm) or a missing row permutation changes it."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests import residuals

D = 2.0 ** -40          # the perturbation


def _rf_case():
    # A = [[0, 3], [4, 0]]: partial pivoting swaps the rows (ipiv = [1, 1]),
    # P A = [[4, 0], [0, 3]] = L U with L = I, U = P A.  Perturbed packed
    # factor U = [[4, 3D], [0, 3 + 4D]]: P A - L U = [[0, -3D], [0, -4D]],
    # ||.||_F = 5D, ||A||_F = 5, n = 2:  R_f = 5D / (5 * 2 * 2^-53) = D 2^52 = 4096.
    A = np.array([[0.0, 3.0], [4.0, 0.0]], order="F")
    LU = np.array([[4.0, 3 * D], [0.0, 3.0 + 4 * D]], order="F")
    ipiv = np.array([1, 1], dtype=np.int32)
    return A, LU, ipiv


def test_r_factor_hand_value():
    A, LU, ipiv = _rf_case()
    assert oracle.r_factor(A, LU, ipiv) == 4096.0


def test_r_factor_exact_factor_is_zero():
    A, LU, ipiv = _rf_case()
    LU[0, 1] = 0.0
    LU[1, 1] = 3.0
    assert oracle.r_factor(A, LU, ipiv) == 0.0


def test_torch_factor_residual_hand_value():
    torch = pytest.importorskip("torch")
    A, LU, ipiv = _rf_case()
    r = residuals.factor_residual(torch.from_numpy(A), torch.from_numpy(LU.copy()), ipiv)
    assert r == 4096.0
    # slabs narrower than the matrix give the same value
    r1 = residuals.factor_residual(torch.from_numpy(A), torch.from_numpy(LU.copy()), ipiv, slab=1)
    assert r1 == 4096.0


def test_r_hpl_hand_value():
    # A = [[3, 1], [2, 1]]: ||A||_inf = 4 (the 1-norm would be 5); b = A [1, 1]^T
    # = [4, 3]; x = [1, 1 + D]: A x - b = [D, D], ||x||_inf = 1 + D, ||b||_inf = 4.
    # R_hpl = D / (2^-53 (4 (1 + D) + 4) 2) exactly, about 512.
    A = np.array([[3.0, 1.0], [2.0, 1.0]], order="F")
    b = np.array([4.0, 3.0])
    x = np.array([1.0, 1.0 + D])
    d = Fraction(D)
    want = d / (Fraction(1, 2 ** 53) * (4 * (1 + d) + 4) * 2)
    got = oracle.r_hpl(A, x, b)
    assert got == pytest.approx(float(want), rel=1e-15)
    assert 511.0 < got < 512.0


def test_r_chol_hand_value():
    # A = [[4, 2], [2, 5]] = L L^T with L = [[2, 0], [1, 2]].  Perturbed
    # L[1,1] = 2 + D: (L L^T)[1,1] = 1 + (2 + D)^2 = 5 + 4D (the D^2 term is
    # below the rounding of 5), so ||A - L L^T||_F = 4D, ||A||_F = 7, n = 2:
    # R_chol = 4D / (7 * 2 * 2^-53) = 2^55 D / 14 = 2^14 / 7.  The strictly upper triangle
    # of the factor array is not part of L and must be ignored.
    A = np.array([[4.0, 2.0], [2.0, 5.0]], order="F")
    F = np.array([[2.0, 99.0], [1.0, 2.0 + D]], order="F")
    got = oracle.r_chol(A, F)
    assert got == pytest.approx(2.0 ** 14 / 7.0, rel=1e-15)


def test_kappa_estimate_matches_exact_condition_number():
    """The Hager estimate used as the yardstick of the full-size FP32
    refinement test, on small matrices where kappa_inf is computed exactly:
    never above it, and within the factor 3 the test allows."""
    import torch
    from tests.test_gpu_ir import _kappa_inf_estimate
    rng = np.random.default_rng(3)
    for n in (50, 200, 400):
        for scale in (None, 1e-3):
            A = rng.uniform(-1, 1, (n, n))
            if scale is not None:
                A[:, 0] *= scale                       # ill-conditioned by a column scaling
            exact = np.linalg.norm(A, np.inf) * np.linalg.norm(np.linalg.inv(A), np.inf)
            est = _kappa_inf_estimate(torch.from_numpy(A))
            assert est <= exact * (1 + 1e-10)
            assert est >= exact / 3.0, (n, scale, est, exact)
