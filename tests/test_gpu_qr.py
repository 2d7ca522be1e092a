"""Householder QR with look-ahead on the GPU (qr_factor / qr_factor_ex) against
the CPU QR oracle element by element (R, the reflector vectors and tau) where
the oracle runs in seconds, bitwise schedule invariance, and at n = 8192 the
property R^T R = A^T A (the Cholesky relation of the Gram matrix)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _qr(gpu, A_np, b, depth, cus=16, lda=None):
    import torch
    m, n = A_np.shape
    dA = gpu.to_device(np.asarray(A_np), lda=lda)
    tau = torch.zeros(max(n, 1), dtype=torch.float64, device="cuda")
    assert gpu.qr_factor(dA, tau, sched=(b, depth, cus)) == 0
    torch.cuda.synchronize()
    assert gpu.lu_factor_info() == (0, 0)
    return gpu.to_host(dA), tau.cpu().numpy()[:n]


@pytest.mark.parametrize("m,n,b,depth,cus,lda", [(1, 1, 32, 1, 16, None), (37, 37, 32, 0, 8, 40),
                                                 (300, 300, 64, 2, 16, None), (1000, 1000, 128, 1, 32, None),
                                                 (1000, 1000, 256, 2, 16, 1003), (700, 500, 64, 2, 16, None),
                                                 (2000, 2000, 128, 2, 32, None), (2500, 2500, 256, 0, 8, None)])
def test_qr_matches_oracle(gpu, m, n, b, depth, cus, lda):
    A = synth.uniform(m, seed=m + n + b)[:, :n].copy(order="F")
    F, tau = _qr(gpu, A, b, depth, cus, lda=lda)
    oF, otau = oracle.geqrf(A, nthreads=8)
    scale = max(1.0, np.abs(np.triu(oF)).max())
    assert np.abs(F - oF).max() <= 1e-11 * scale
    assert np.abs(tau - otau).max() <= 1e-11


@pytest.mark.parametrize("m,n,b,depth", [(9000, 200, 128, 2), (20000, 300, 64, 1)])
def test_qr_tall_skinny_matches_oracle(gpu, m, n, b, depth):
    """Panels of 9 and 20 work-groups: the cross-group sums against the oracle."""
    A = synth.rhs(m, seed=m + n, nrhs=n)
    F, tau = _qr(gpu, A, b, depth, 32)
    oF, otau = oracle.geqrf(A, nthreads=8)
    scale = max(1.0, np.abs(np.triu(oF)).max())
    assert np.abs(F - oF).max() <= 1e-11 * scale
    assert np.abs(tau - otau).max() <= 1e-11


def test_qr_schedule_invariance_bitwise(gpu):
    A = synth.uniform(2600, seed=31)
    ref = None
    for depth in (0, 1, 2):
        for cus in (8, 16, 32):
            F, tau = _qr(gpu, A, 128, depth, cus)
            if ref is None:
                ref = (F, tau)
            else:
                assert np.array_equal(F, ref[0]) and np.array_equal(tau, ref[1]), (depth, cus)


def test_qr_argument_errors(gpu):
    import torch
    dA = gpu.to_device(np.eye(4, order="F"))
    tau = torch.zeros(4, dtype=torch.float64, device="cuda")
    lib = gpu.load()
    p, t = dA.data_ptr(), tau.data_ptr()
    assert lib.qr_factor(-1, 1, p, 4, t, None) == -1
    assert lib.qr_factor(3, 4, p, 4, t, None) == -2
    assert lib.qr_factor(4, 4, None, 4, t, None) == -3
    assert lib.qr_factor(4, 4, p, 3, t, None) == -4
    assert lib.qr_factor(4, 4, p, 4, None, None) == -5
    assert gpu.qr_factor(dA, tau, sched=(512, 1, 16)) == -6
    assert lib.qr_factor(0, 0, None, 1, None, None) == 0


@pytest.mark.timeout(600)
def test_qr_8192_gram_relation(gpu):
    """R^T R = A^T A at full scale: ||R^T R - A^T A||_F / ||A^T A||_F small."""
    import torch
    n = 8192
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    A0 = gpu.colmajor(n)
    A0.uniform_(-1.0, 1.0, generator=g)
    torch.cuda.synchronize()
    F = A0.clone()
    tau = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert gpu.qr_factor(F, tau) == 0
    torch.cuda.synchronize()
    assert gpu.lu_factor_info() == (0, 0)
    R = torch.triu(F)
    G = A0.t() @ A0
    E = R.t() @ R - G
    rel = (torch.linalg.norm(E) / torch.linalg.norm(G)).item()
    assert rel <= 1e-12, rel
    assert bool(torch.isfinite(tau).all()) and bool(((tau >= 0) & (tau <= 2)).all())
