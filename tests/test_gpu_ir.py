"""Mixed-precision factorization + FP64 iterative refinement (lu_solve_ir) on
the GPU: the refined solution meets the HPL acceptance test, agrees with the
oracle's FP64 solution within the conditioning bound, and falls back to an
FP64 factorization when refinement cannot converge."""
import os

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
@pytest.mark.parametrize("n", [2048, 1000, 777])  # 777: 13 blocks of the FP32 solves, the last pair one block
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


def test_ir_singular_matrix_reported(gpu):
    """A zero column makes the FP64 factor singular (INFO = its index + 1): the
    plain FP64 path and the mixed path (whose fall-back refactors in FP64)
    return LU_ERR_SINGULAR and a NaN residual instead of a solution."""
    A = synth.uniform(300, seed=13)
    A[:, 41] = 0.0
    b = synth.rhs(300, seed=13)[:, 0]
    for prec in (gpu.LU_FP64, gpu.LU_MIXED_FP16, gpu.LU_FP32):
        st, it, res, _ = _ir(gpu, A, b, prec)
        assert st == gpu.LU_ERR_SINGULAR, (prec, st)
        assert np.isnan(res)


# ---- full size (n = 32768), against the oracle's cached FP64 solution -------

def _xo(workload):
    """The oracle's solution of the seed-1 n = 32768 system of `workload`,
    written by tests/golden/make_xo.py, and its metadata."""
    import json
    from tests.golden import make_xo
    npy, js = make_xo.paths(workload, 32768, 1)
    if not os.path.exists(npy):
        pytest.fail("oracle solution %s missing: run tests/golden/make_xo.py %s" % (npy, workload))
    with open(js) as f:
        meta = json.load(f)
    return np.load(npy), meta


_BIG = {}


def _big_system(gpu, workload):
    """Seeded n = 32768 system on the device, checked against the fingerprint
    of the matrix the oracle solved (kept for the module: 8.6 GB each)."""
    import torch
    from tests.golden import make_xo
    if workload not in _BIG:
        xo, meta = _xo(workload)
        A = make_xo.make_matrix(workload, 32768, 1)
        assert make_xo.check_fingerprint(A, meta["fingerprint"]), "regenerated matrix differs"
        dA = gpu.to_device(A)
        del A
        b = synth.rhs(32768, seed=1)[:, 0]
        _BIG.clear()
        _BIG[workload] = (dA, torch.from_numpy(b).cuda(), xo, meta)
        torch.cuda.synchronize()
    return _BIG[workload]


def _check_full_size_ir(gpu, workload, prec, kappa):
    import torch
    n = 32768
    dA, dB, xo, meta = _big_system(gpu, workload)
    dX = torch.zeros(n, dtype=torch.float64, device="cuda")
    print("case", workload, prec, flush=True)
    st, it, res = gpu.lu_solve_ir(dA, dB, dX, prec=prec, max_iter=20)
    torch.cuda.synchronize()
    assert st == gpu.LU_IR_OK and 1 <= it <= 20, (st, it, res)
    # the HPL residual recomputed with torch's FP64 matrix-vector product
    r = torch.mv(dA, dX) - dB
    anorm = dA.abs().sum(dim=1).max().item()
    rh = r.abs().max().item() / (EPS * (anorm * dX.abs().max().item() + dB.abs().max().item()) * n)
    assert rh <= 16.0
    assert abs(rh - res) <= 1.0 + 2.0 / n       # evaluation rounding of b - A x, as above
    # forward error against the oracle: both solutions pass the HPL test, so
    # ||x - x_o|| / ||x_o|| <= 2 * 16 * n * eps * kappa_inf(A)
    x = dX.cpu().numpy()
    err = np.abs(x - xo).max() / np.abs(xo).max()
    assert err <= 2 * 16 * n * EPS * kappa, err
    return it, err


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [2, 3])         # FP16 and BF16 trailing updates
def test_mixed_ir_n32768_against_oracle(gpu, prec):
    """C4(a) at full size: FP16/BF16 trailing GEMM, FP32 panel and TRSM, FP64
    refinement on the row-dominant matrix.  Its kappa_inf is about 2 (A = D + R
    with D = diag of about n/2 and R of random signs, ||D^-1 R||_2 ~ 4/sqrt(n));
    the bound uses 4."""
    _check_full_size_ir(gpu, "dominant", prec, kappa=4.0)


def _kappa_inf_estimate(dA):
    """Estimate of kappa_inf(A) = ||A||_inf ||A^-1||_inf: Hager's 1-norm
    estimator (Higham, Accuracy and Stability of Numerical Algorithms, Alg.
    15.4) applied to B = A^-T, whose 1-norm is ||A^-1||_inf, with torch's own
    LU (a yardstick independent of this library).  The estimate is a lower
    bound, in practice within a factor of 3."""
    import torch
    n = dA.shape[0]
    LUt, piv = torch.linalg.lu_factor(dA)
    x = torch.full((n, 1), 1.0 / n, dtype=torch.float64, device=dA.device)
    est = 0.0
    for it in range(5):
        y = torch.linalg.lu_solve(LUt, piv, x, adjoint=True)        # B x = A^-T x
        est = max(est, y.abs().sum().item())
        xi = torch.where(y >= 0, 1.0, -1.0).to(torch.float64)
        z = torch.linalg.lu_solve(LUt, piv, xi)                      # B^T xi = A^-1 xi
        zmax, j = z.abs().max(dim=0)
        if it > 0 and zmax.item() <= (z * x).sum().item():
            break
        x = torch.zeros_like(x)
        x[j.item(), 0] = 1.0
    del LUt, piv
    anorm = dA.abs().sum(dim=1).max().item()
    return anorm * est


@pytest.mark.timeout(900)
def test_fp32_ir_n32768_against_oracle(gpu):
    """C4(b) at full size: FP32 LU of the non-dominant uniform matrix, FP64
    refinement.  Both the refined solution and the oracle's pass the HPL test
    (normwise backward error at most 16 n eps each), so their difference is
    bounded by 2 kappa_inf(A) 16 n eps to first order; kappa_inf comes from
    Hager's estimator, taken 3 times over for its underestimation.  The FP64
    LU solution's error is printed beside it: refinement stops at the HPL
    test, so its forward error may exceed the FP64 LU's."""
    import torch
    n = 32768
    dA, dB, xo, meta = _big_system(gpu, "uniform")
    kappa = _kappa_inf_estimate(dA)
    torch.cuda.empty_cache()
    LU = dA.clone()
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert gpu.lu_factor_ex(LU, ipiv, prec=gpu.LU_FP64) == 0
    x64 = dB.clone().reshape(n, 1)
    assert gpu.lu_solve_ex(LU, ipiv, x64) == 0
    torch.cuda.synchronize()
    del LU
    e64 = np.abs(x64.cpu().numpy()[:, 0] - xo).max() / np.abs(xo).max()
    it, err = _check_full_size_ir(gpu, "uniform", gpu.LU_FP32, kappa=3.0 * kappa)
    print("fp32+IR n=32768: kappa_inf estimate %.3e, iterations %d, error %.3e (FP64 LU error %.3e)" % (
        kappa, it, err, e64))
