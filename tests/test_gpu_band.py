"""Two-sided band reduction on the GPU (band_reduce) against the CPU band
oracle element by element (band, column and row reflectors, tauq, taup) where
the oracle runs in seconds, including ragged last panels, w >= n, the widest
band (384) and a padded lda; at larger n the orthogonal invariants (singular
values, Frobenius norm) and the first column panel against qr_factor."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _band(gpu, A_np, w, lda=None):
    import torch
    n = A_np.shape[0]
    dA = gpu.to_device(np.asarray(A_np), lda=lda)
    tq = torch.zeros(max(n, 1), dtype=torch.float64, device="cuda")
    tp = torch.full((max(n, 1),), 7.0, dtype=torch.float64, device="cuda")   # must come back zeroed where unused
    assert gpu.band_reduce(dA, w, tq, tp) == 0
    torch.cuda.synchronize()
    assert gpu.lu_factor_info() == (0, 0)
    return gpu.to_host(dA), tq.cpu().numpy()[:n], tp.cpu().numpy()[:n]


@pytest.mark.parametrize("n,w,lda", [(1, 1, None), (37, 8, 40), (300, 32, None), (500, 64, None),
                                     (700, 128, None), (257, 300, None), (640, 384, None), (900, 96, 903)])
def test_band_matches_oracle(gpu, n, w, lda):
    A = synth.uniform(n, seed=n + 3 * w)
    F, tq, tp = _band(gpu, A, w, lda=lda)
    oF, otq, otp = oracle.gebrd_band(A, w)
    scale = max(1.0, np.abs(oracle.band_part(oF, w)).max())
    assert np.abs(F - oF).max() <= 1e-11 * scale
    assert np.abs(tq - otq).max() <= 1e-11
    assert np.abs(tp - otp).max() <= 1e-11


def test_band_2048_singular_values(gpu):
    n, w = 2048, 128
    A = synth.uniform(n, seed=21)
    F, _, _ = _band(gpu, A, w)
    sa = np.linalg.svd(A, compute_uv=False)
    sb = np.linalg.svd(oracle.band_part(F, w), compute_uv=False)
    assert np.abs(sa - sb).max() <= 1e-12 * sa[0]


def test_band_8192_invariants(gpu):
    """||B||_F = ||A||_F, and the first column panel is the Householder QR of
    A[:, :w] (the same panel launch as qr_factor with b = w: bitwise)."""
    import torch
    n, w = 8192, 128
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    A0 = gpu.colmajor(n)
    A0.uniform_(-1.0, 1.0, generator=g)
    torch.cuda.synchronize()
    F = A0.clone()
    tq = torch.zeros(n, dtype=torch.float64, device="cuda")
    tp = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert gpu.band_reduce(F, w, tq, tp) == 0
    torch.cuda.synchronize()
    assert gpu.lu_factor_info() == (0, 0)
    i = torch.arange(n, device="cuda")
    off = i[None, :] - i[:, None]
    B = torch.where((off >= 0) & (off <= w), F, torch.zeros((), dtype=F.dtype, device="cuda"))
    na, nb = torch.linalg.norm(A0).item(), torch.linalg.norm(B).item()
    assert abs(na - nb) <= 1e-12 * na
    P = A0[:, :w].clone()
    tqr = torch.zeros(w, dtype=torch.float64, device="cuda")
    assert gpu.qr_factor(P, tqr, sched=(128, 0, 0)) == 0
    torch.cuda.synchronize()
    assert torch.equal(P, F[:, :w]) and torch.equal(tqr, tq[:w])
    assert bool(torch.isfinite(tp).all()) and bool(((tp >= 0) & (tp <= 2)).all())


def test_band_argument_errors(gpu):
    import torch
    dA = gpu.to_device(np.eye(4, order="F"))
    t = torch.zeros(4, dtype=torch.float64, device="cuda")
    lib = gpu.load()
    p, tp = dA.data_ptr(), t.data_ptr()
    assert lib.band_reduce(-1, p, 4, 2, tp, tp, None) == -1
    assert lib.band_reduce(4, None, 4, 2, tp, tp, None) == -2
    assert lib.band_reduce(4, p, 3, 2, tp, tp, None) == -3
    assert lib.band_reduce(4, p, 4, 0, tp, tp, None) == -4
    assert lib.band_reduce(4, p, 4, 385, tp, tp, None) == -4
    assert lib.band_reduce(4, p, 4, 2, None, tp, None) == -5
    assert lib.band_reduce(4, p, 4, 2, tp, None, None) == -6
    assert lib.band_reduce(0, None, 1, 2, None, None, None) == 0
