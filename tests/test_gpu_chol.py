"""Cholesky with look-ahead on the GPU (chol_factor / chol_factor_ex) against
the CPU Cholesky oracle, element by element where the oracle runs in seconds,
and by properties that hold at any size (scaled residual, untouched upper
triangle, bitwise invariance over schedules)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _chol(gpu, A_np, b, depth, panel_cus=16, lda=None):
    import torch
    dA = gpu.to_device(np.asarray(A_np), lda=lda)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert gpu.chol_factor_ex(dA, sched=(b, depth, panel_cus), d_info=info) == 0
    torch.cuda.synchronize()
    assert gpu.lu_factor_info()[0] == 0
    return gpu.to_host(dA), int(info.item())


@pytest.mark.parametrize("n,b,depth,cus,lda", [(1, 64, 1, 16, None), (37, 32, 0, 8, 40), (300, 64, 2, 16, None),
                                               (1000, 128, 1, 32, None), (1000, 256, 2, 16, 1003),
                                               (1536, 512, 2, 32, None), (2000, 256, 0, 8, None),
                                               (2500, 256, 2, 32, None), (4096, 256, 2, 8, None),
                                               (4096, 128, 1, 16, None)])
def test_chol_matches_oracle(gpu, n, b, depth, cus, lda):
    A = synth.spd(n, seed=n + b)
    F, info = _chol(gpu, A, b, depth, cus, lda=lda)
    oF, oinfo = oracle.potrf(A, nthreads=8)
    assert info == oinfo == 0
    L, oL = np.tril(F), np.tril(oF)
    assert np.abs(L - oL).max() <= 1e-12 * np.abs(oL).max()
    assert oracle.r_chol(A, F) <= 16.0


def test_upper_triangle_and_padding_untouched(gpu):
    import torch
    n, lda = 700, 709
    A = synth.spd(n, seed=11)
    Au = A.copy(order="F")
    Au[np.triu_indices(n, 1)] = 12345.0          # never read: the factor comes from the lower triangle
    dA = gpu.to_device(Au, lda=lda)
    full = torch.as_strided(dA, (lda, n), (1, lda))
    full[n:, :] = -777.0
    assert gpu.chol_factor_ex(dA, sched=(128, 2, 16)) == 0
    torch.cuda.synchronize()
    F = gpu.to_host(dA)
    assert np.array_equal(np.triu(F, 1), np.triu(Au, 1))
    assert bool((full[n:, :] == -777.0).all())
    oF, _ = oracle.potrf(A)
    assert np.abs(np.tril(F) - np.tril(oF)).max() <= 1e-12 * np.abs(np.tril(oF)).max()


@pytest.mark.parametrize("bad", [0, 150, 299])
def test_not_positive_definite_info(gpu, bad):
    A = synth.spd(300, seed=5)
    A[bad, bad] = -1.0
    _, oinfo = oracle.potrf(A)
    assert oinfo > 0
    _, info = _chol(gpu, A, 64, 2)
    assert info == oinfo


# the lower solve takes 64-row blocks two per work-group: 191 and 4160 give an
# odd block count (a work-group with one block) past the first pair
@pytest.mark.parametrize("n,nrhs,lda,ldb", [(1, 1, None, None), (37, 2, 40, 41), (1000, 1, None, None),
                                            (1500, 3, 1503, 1500), (191, 2, 193, None), (4160, 1, None, None)])
def test_chol_solve_matches_oracle(gpu, n, nrhs, lda, ldb):
    import torch
    from scipy.linalg import solve_triangular
    A = synth.spd(n, seed=n + 3)
    B = synth.rhs(n, seed=n + 3, nrhs=nrhs)
    dA = gpu.to_device(A, lda=lda)
    assert gpu.chol_factor_ex(dA, sched=(128, 2, 16)) == 0
    dB = gpu.to_device(B, lda=ldb)
    assert gpu.chol_solve(dA, dB) == 0
    torch.cuda.synchronize()
    X = gpu.to_host(dB)
    oF, _ = oracle.potrf(A)
    oL = np.tril(oF)
    Xo = solve_triangular(oL.T, solve_triangular(oL, B, lower=True), lower=False)
    assert np.abs(X - Xo).max() <= 1e-10 * max(1.0, np.abs(Xo).max())
    for c in range(nrhs):
        assert oracle.r_hpl(A, X[:, c], B[:, c]) <= 16.0


def test_chol_solve_argument_errors(gpu):
    dA = gpu.to_device(np.eye(4, order="F"))
    lib = gpu.load()
    p = dA.data_ptr()
    assert lib.chol_solve(-1, 1, p, 4, p, 4, None) == -1
    assert lib.chol_solve(4, -1, p, 4, p, 4, None) == -2
    assert lib.chol_solve(4, 1, None, 4, p, 4, None) == -3
    assert lib.chol_solve(4, 1, p, 3, p, 4, None) == -4
    assert lib.chol_solve(4, 1, p, 4, None, 4, None) == -5
    assert lib.chol_solve(4, 1, p, 4, p, 3, None) == -6
    assert lib.chol_solve(0, 1, None, 1, None, 1, None) == 0


def test_zero_matrix_info(gpu):
    _, info = _chol(gpu, np.zeros((100, 100), order="F"), 32, 1)
    assert info == 1


def test_chol_schedule_invariance_bitwise(gpu):
    n, b = 1500, 128
    A = synth.spd(n, seed=21)
    ref = None
    for depth in (0, 1, 2):
        for cus in (8, 16, 32):
            F, _ = _chol(gpu, A, b, depth, cus)
            if ref is None:
                ref = F
            else:
                assert np.array_equal(F, ref), (depth, cus)


def test_chol_argument_errors(gpu):
    import torch
    dA = gpu.to_device(np.eye(4, order="F"))
    assert gpu.chol_factor_ex(dA, sched=(100, 1, 16)) == -4
    assert gpu.chol_factor_ex(dA, sched=(64, 3, 16)) == -4
    assert gpu.load().chol_factor(-1, dA.data_ptr(), 4, None) == -1
    assert gpu.load().chol_factor(4, None, 4, None) == -2
    assert gpu.load().chol_factor(4, dA.data_ptr(), 3, None) == -3
    assert gpu.load().chol_factor(0, None, 1, None) == 0
    torch.cuda.synchronize()


def _device_spd(gpu, n, seed):
    """SPD matrix built on the device like synth.spd: (B + B^T)/2, diagonal =
    row absolute sum (the full-size workload; no host copy needed)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    A = gpu.colmajor(n)
    A.uniform_(-1.0, 1.0, generator=g)
    for c0 in range(0, n, 4096):                 # symmetrize in slabs: A[i, j] = A[j, i] = mean
        c1 = min(n, c0 + 4096)
        blk = A[c0:c1, :].clone()
        sym = (blk + A[:, c0:c1].t()) / 2.0
        A[c0:c1, :] = sym
        A[:, c0:c1] = sym.t()
    rs = A.abs().sum(dim=1)
    A.diagonal().copy_(rs)
    return A


@pytest.mark.timeout(900)
def test_chol_32768_residual(gpu):
    """Full-size FP64 Cholesky with look-ahead: scaled residual ||A - L L^T||_F /
    (||A||_F n eps) with a library GEMM in column slabs, positive diagonal."""
    import torch
    n = 32768
    A0 = _device_spd(gpu, n, 7)
    assert torch.equal(A0[:4096, :4096], A0[:4096, :4096].t())
    F = A0.clone()
    assert gpu.chol_factor(F) == 0
    torch.cuda.synchronize()
    assert gpu.lu_factor_info() == (0, 0)
    L = torch.tril(F)
    assert bool((L.diagonal() > 0).all())
    acc = 0.0
    for c0 in range(0, n, 4096):
        c1 = min(n, c0 + 4096)
        R = torch.tril(A0[:, c0:c1], diagonal=-c0) - L[:, :c1] @ L[c0:c1, :c1].t()
        R = torch.tril(R, diagonal=-c0)             # compare the lower triangle only
        acc += float((R * R).sum().item())
        del R
    nA = float((torch.tril(A0) ** 2).sum().item()) ** 0.5
    rf = acc ** 0.5 / (nA * n * 2.0 ** -53)
    assert rf <= 16.0, rf
    del L
    # solve with the factor: HPL residual of A x = b with A applied by a library GEMV
    g = torch.Generator(device="cuda")
    g.manual_seed(8)
    b = torch.empty(n, dtype=torch.float64, device="cuda").uniform_(-1.0, 1.0, generator=g)
    x = b.clone()
    assert gpu.chol_solve(F, x) == 0
    torch.cuda.synchronize()
    r = (A0 @ x - b).abs().max().item()
    hpl = r / (2.0 ** -53 * (A0.abs().sum(dim=1).max().item() * x.abs().max().item() + b.abs().max().item()) * n)
    assert hpl <= 16.0, hpl
