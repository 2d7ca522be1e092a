"""Mixed-precision factorization + FP64 iterative refinement (lu_solve_ir) on
the GPU: the refined solution meets the HPL acceptance test, agrees with the
oracle's FP64 solution within the conditioning bound, and falls back to an
FP64 factorization when refinement cannot converge."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53


def _ir(gpu, A, b, prec, max_iter=10, lda=None):
    import torch
    n = A.shape[0]
    dA = gpu.to_device(A, lda=lda)
    dB = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    dX = torch.zeros(n, dtype=torch.float64, device="cuda")
    A_before = dA.clone()
    st, it, res = gpu.lu_solve_ir(dA, dB, dX, prec=prec, max_iter=max_iter)
    torch.cuda.synchronize()
    assert torch.equal(dA.view(torch.int64), A_before.view(torch.int64)), "lu_solve_ir must not modify A"
    return st, it, res, dX.cpu().numpy()


def _forward_error_bound(A, n):
    # HPL acceptance residual 16 and kappa_inf(A) bound the forward error:
    # ||x - x_o|| / ||x_o|| <= 2 * 16 * n * eps * kappa (both solutions pass the test)
    kappa = np.linalg.cond(A, np.inf)
    return 2 * 16 * n * EPS * kappa


@pytest.mark.parametrize("prec", [2, 3])          # LU_MIXED_FP16, LU_MIXED_BF16
@pytest.mark.parametrize("n", [2048, 1000])
def test_half_precision_ir_on_dominant_matrix(gpu, prec, n):
    A = synth.dominant(n, seed=5)
    b = synth.rhs(n, seed=5)[:, 0]
    st, it, res, x = _ir(gpu, A, b, prec)
    assert st == gpu.LU_IR_OK, (st, it, res)
    assert 1 <= it <= 10
    r = oracle.r_hpl(A, x, b)
    # the library's own residual may differ from this one by the rounding of
    # evaluating b - A x in FP64, at most (n+1) eps (|b| + |A||x|): ~1 in these units
    assert r <= 16.0 and abs(r - res) <= 1.0 + 2.0 / n
    xo = oracle.solve(A, b, nthreads=8)
    err = np.abs(x - xo).max() / np.abs(xo).max()
    assert err <= _forward_error_bound(A, n), err


@pytest.mark.parametrize("n", [2048, 777])
def test_fp32_ir_on_uniform_matrix(gpu, n):
    A = synth.uniform(n, seed=7)
    b = synth.rhs(n, seed=7)[:, 0]
    st, it, res, x = _ir(gpu, A, b, gpu.LU_FP32)
    assert st == gpu.LU_IR_OK, (st, it, res)
    r = oracle.r_hpl(A, x, b)
    assert r <= 16.0
    xo = oracle.solve(A, b, nthreads=8)
    err = np.abs(x - xo).max() / np.abs(xo).max()
    assert err <= _forward_error_bound(A, n), err


def test_ir_falls_back_to_fp64_when_not_converged(gpu):
    # one FP32 refinement step cannot reach the FP64 test on an ill-conditioned
    # uniform matrix (kappa ~ 1e5: first residual ~ 2^-24 kappa / (n eps) >> 16)
    n = 1024
    A = synth.uniform(n, seed=9)
    b = synth.rhs(n, seed=9)[:, 0]
    st, it, res, x = _ir(gpu, A, b, gpu.LU_FP32, max_iter=1)
    assert st == gpu.LU_IR_FELL_BACK
    assert oracle.r_hpl(A, x, b) <= 16.0


def test_ir_fp64_path_and_lda(gpu):
    n = 600
    A = synth.uniform(n, seed=11)
    b = synth.rhs(n, seed=11)[:, 0]
    st, it, res, x = _ir(gpu, A, b, gpu.LU_FP64, lda=611)
    assert st == gpu.LU_IR_OK
    assert oracle.r_hpl(A, x, b) <= 16.0


def test_ir_rejects_nonfinite_input(gpu):
    A = synth.dominant(256, seed=2)
    A[17, 3] = np.nan
    b = synth.rhs(256, seed=2)[:, 0]
    st, _, _, _ = _ir(gpu, A, b, 2)
    assert st == gpu.LU_ERR_NONFINITE
    A = synth.dominant(256, seed=2)
    b[5] = np.inf
    st, _, _, _ = _ir(gpu, A, b, 2)
    assert st == gpu.LU_ERR_NONFINITE


@pytest.mark.timeout(600)
def test_mixed_fp16_ir_n32768(gpu):
    """C4(a) at full size: FP16 trailing GEMM, FP32 panel/TRSM, FP64 refinement.
    The residual is recomputed independently with torch's FP64 matrix-vector
    product; the oracle's solution is out of reach at this size."""
    import torch
    n = 32768
    A = synth.dominant(n, seed=1)
    b = synth.rhs(n, seed=1)[:, 0]
    dA = gpu.to_device(A)
    del A
    dB = torch.from_numpy(b).cuda()
    dX = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, it, res = gpu.lu_solve_ir(dA, dB, dX, prec=2, max_iter=10)
    torch.cuda.synchronize()
    assert st == gpu.LU_IR_OK and it <= 10
    r = torch.mv(dA, dX) - dB
    anorm = dA.abs().sum(dim=1).max().item()
    rh = r.abs().max().item() / (EPS * (anorm * dX.abs().max().item() + dB.abs().max().item()) * n)
    assert rh <= 16.0
    assert abs(rh - res) <= 1.0 + 2.0 / n       # evaluation rounding of b - A x, as above
