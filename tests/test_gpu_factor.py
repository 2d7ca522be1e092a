"""End-to-end parity of lu_factor / lu_factor_ex / lu_solve on the GPU against
the CPU oracle (element by element where the oracle runs in seconds) and
against properties that hold at any size (scaled residuals, planted factors)."""
import numpy as np
import pytest

import oracle
import synth
from tests import pins, residuals

pytestmark = pytest.mark.gpu


def _factor(gpu, A_np, b, depth, panel_cus=16, prec=0, lda=None, taper=-1):
    """Factor on the GPU; taper -1 (default here) keeps every panel b wide, so
    that each test exercises the block size it names."""
    import torch
    n = A_np.shape[0]
    dt = torch.float64 if prec == 0 else torch.float32
    dA = gpu.to_device(np.asarray(A_np), dt, lda=lda)
    ipiv = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = gpu.lu_factor_ex(dA, ipiv, prec=prec, sched=(b, depth, panel_cus, taper), d_info=info)
    assert rc == 0
    torch.cuda.synchronize()
    rc2, _ = gpu.lu_factor_info()
    assert rc2 == 0
    return gpu.to_host(dA).astype(np.float64), ipiv.cpu().numpy()[:n], int(info.item())


def test_512_b64_depth0_matches_oracle(gpu):
    A = synth.uniform(512, seed=1)
    LU, ipiv, info = _factor(gpu, A, 64, 0)
    oLU, oip, oinfo = oracle.getrf(A, nthreads=8)
    assert info == oinfo == 0
    assert np.array_equal(ipiv, oip)
    assert np.abs(LU - oLU).max() <= 1e-12 * np.abs(oLU).max()
    assert oracle.r_factor(A, LU, ipiv) <= 16.0


@pytest.mark.parametrize("n,b,depth,lda", [(1000, 64, 1, None), (1000, 128, 2, 1003), (1, 64, 1, None),
                                           (37, 64, 0, 40), (65, 32, 2, None), (777, 256, 1, None),
                                           (1536, 512, 2, None), (300, 128, 0, 301)])
def test_ragged_and_schedules_match_oracle(gpu, n, b, depth, lda):
    A = synth.uniform(n, seed=n + b)
    LU, ipiv, info = _factor(gpu, A, b, depth, lda=lda)
    oLU, oip, _ = oracle.getrf(A, nthreads=8)
    gap_ok = True
    assert np.array_equal(ipiv, oip) or not gap_ok
    assert np.abs(LU - oLU).max() <= 1e-11 * max(1.0, np.abs(oLU).max())
    assert oracle.r_factor(A, LU, ipiv) <= 16.0


def test_lda_padding_untouched(gpu):
    import torch
    n, lda = 300, 311
    A = synth.uniform(n, seed=3)
    dA = gpu.to_device(A, lda=lda)
    base = dA.t()  # (n, lda) storage view
    full = torch.as_strided(dA, (lda, n), (1, lda))
    full[n:, :] = 12345.0
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert gpu.lu_factor(dA, ipiv) == 0
    torch.cuda.synchronize()
    assert bool((full[n:, :] == 12345.0).all())
    del base


def test_schedule_invariance_bitwise(gpu):
    n, b = 1500, 128
    A = synth.uniform(n, seed=21)
    ref = None
    for depth in (0, 1, 2):
        for cus in (8, 16, 32):
            LU, ipiv, _ = _factor(gpu, A, b, depth, cus)
            if ref is None:
                ref = (LU, ipiv)
            else:
                assert np.array_equal(LU, ref[0]) and np.array_equal(ipiv, ref[1]), (depth, cus)


@pytest.mark.parametrize("n,b,depth", [(3000, 256, 2), (2100, 512, 1), (1000, 128, 0)])
def test_taper_matches_oracle(gpu, n, b, depth):
    """Early-termination taper (panels narrowing to 128 columns once the
    trailing matrix is small): the same factorization as the oracle's."""
    A = synth.uniform(n, seed=n + 7)
    LU, ipiv, info = _factor(gpu, A, b, depth, taper=1)
    oLU, oip, oinfo = oracle.getrf(A, nthreads=8)
    assert info == oinfo == 0
    assert np.array_equal(ipiv, oip)
    assert np.abs(LU - oLU).max() <= 1e-11 * max(1.0, np.abs(oLU).max())


def test_taper_schedule_invariance_bitwise(gpu):
    """With the taper, panel widths 256 -> 128 are fixed by n and the
    precision, so depth and CU share leave every bit of the result unchanged."""
    import torch
    n = 17000
    A = synth.uniform(n, seed=5)
    dA0 = gpu.to_device(A)
    del A
    ref = None
    for depth, cus in ((0, 16), (1, 8), (2, 32)):
        dA = dA0.clone()
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        assert gpu.lu_factor_ex(dA, ipiv, sched=(256, depth, cus, 1)) == 0
        torch.cuda.synchronize()
        assert gpu.lu_factor_info() == (0, 0)
        if ref is None:
            ref = (dA, ipiv)
        else:
            assert torch.equal(dA, ref[0]) and torch.equal(ipiv, ref[1]), (depth, cus)
    rf = _device_residual(gpu, dA0, ref[0], ref[1].cpu().numpy())
    assert rf <= 16.0, rf


def test_mixed_taper_ir(gpu):
    """Mixed-precision LU with the taper (128-wide tail panels, the library
    default), refined to the FP64 acceptance test."""
    import torch
    n = 5000
    A = synth.dominant(n, seed=3)
    b = synth.rhs(n, seed=3)[:, 0]
    dA = gpu.to_device(A)
    dB = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    dX = torch.zeros(n, dtype=torch.float64, device="cuda")
    rc, sch = gpu.lu_schedule_default(n, gpu.LU_MIXED_FP16)
    assert rc == 0 and sch[3] == 1
    st, it, res = gpu.lu_solve_ir(dA, dB, dX, prec=gpu.LU_MIXED_FP16, max_iter=10)
    torch.cuda.synchronize()
    assert st == 0 and res <= 16.0, (st, it, res)
    assert oracle.r_hpl(A, dX.cpu().numpy(), b) <= 16.0


def test_zero_column_and_zero_matrix_info(gpu):
    A = synth.uniform(200, seed=5)
    A[:, 70] = 0.0
    _, _, info = _factor(gpu, A, 64, 1)
    _, _, oinfo = oracle.getrf(A)
    assert info == oinfo == 71
    LU, ipiv, info = _factor(gpu, np.zeros((130, 130), order="F"), 64, 1)
    assert info == 1 and np.array_equal(ipiv, np.arange(130))


def test_identity_and_permutation(gpu):
    n = 257
    LU, ipiv, _ = _factor(gpu, np.eye(n, order="F"), 64, 1)
    assert np.array_equal(LU, np.eye(n)) and np.array_equal(ipiv, np.arange(n))
    perm = synth.rng(9, 2).permutation(n)
    A = np.asfortranarray(np.eye(n)[perm, :])
    LU, ipiv, _ = _factor(gpu, A, 64, 2)
    assert np.array_equal(LU, np.eye(n))
    assert np.array_equal(A[oracle.perm_from_ipiv(ipiv), :], np.eye(n))


@pytest.mark.parametrize("n", [512, 2000])
def test_planted_factors_recovered(gpu, n):
    A, L, U, perm = synth.planted(n, seed=4)
    LU, ipiv, _ = _factor(gpu, A, 128, 1)
    assert np.array_equal(ipiv, pins.planted_ipiv(perm))
    Lh, Uh = oracle.unpack(LU)
    assert np.abs(Lh - L).max() <= 1e-12
    assert np.abs(Uh - U).max() <= 1e-12 * np.abs(U).max()


# the triangular solves take 64-row blocks two per work-group: an odd number of
# blocks (37, 130, 191, 4160) leaves a work-group with one block, and ragged
# sizes a partial block
@pytest.mark.parametrize("n,nrhs", [(512, 1), (2000, 3), (100, 1), (1, 1), (37, 2), (64, 1), (130, 2), (191, 1),
                                    (4160, 1)])
def test_solve_matches_oracle(gpu, n, nrhs):
    import torch
    A = synth.uniform(n, seed=n)
    B = synth.rhs(n, seed=n, nrhs=nrhs)
    LU, ipiv, _ = _factor(gpu, A, 128, 1)
    dLU = gpu.to_device(LU)
    dp = torch.tensor(ipiv, dtype=torch.int32, device="cuda")
    dB = gpu.to_device(B)
    assert gpu.lu_solve_ex(dLU, dp, dB) == 0
    torch.cuda.synchronize()
    X = gpu.to_host(dB)
    oLU, oip, _ = oracle.getrf(A, nthreads=8)
    Xo = oracle.getrs(oLU, oip, B)
    for c in range(nrhs):
        assert oracle.r_hpl(A, X[:, c], B[:, c]) <= 16.0
    assert np.abs(X - Xo).max() <= 1e-8 * np.abs(Xo).max()


def test_solve_leading_dimension_past_2gib(gpu):
    """Columns more than 2^31 bytes apart (lda * 8 * 300 > 2^31): the solve's
    column addresses are formed per column, not as 32-bit offsets from one base."""
    import torch
    n, lda = 300, (1 << 21) + 64
    A = synth.uniform(n, seed=11)
    B = synth.rhs(n, seed=11, nrhs=1)
    LU, ipiv, _ = _factor(gpu, A, 128, 1)
    dLU = gpu.to_device(LU, lda=lda)
    dp = torch.tensor(ipiv, dtype=torch.int32, device="cuda")
    dB = gpu.to_device(B)
    assert gpu.lu_solve_ex(dLU, dp, dB) == 0
    torch.cuda.synchronize()
    X = gpu.to_host(dB)
    oLU, oip, _ = oracle.getrf(A, nthreads=8)
    Xo = oracle.getrs(oLU, oip, B)
    assert np.abs(X - Xo).max() <= 1e-8 * np.abs(Xo).max()
    del dLU
    torch.cuda.empty_cache()


def test_solve_square_default_stream_form(gpu):
    import torch
    n = 333
    A = synth.uniform(n, seed=2)
    b = synth.rhs(n, seed=2)
    dA = gpu.to_device(A)
    dp = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert gpu.lu_factor(dA, dp) == 0
    torch.cuda.synchronize()
    db = gpu.to_device(b)
    assert gpu.lu_solve(dA, dp, db) == 0
    x = gpu.to_host(db)[:, 0]
    assert oracle.r_hpl(A, x, b[:, 0]) <= 16.0


def test_fp32_factor_residual(gpu):
    n = 1000
    A = synth.uniform(n, seed=8)
    LU, ipiv, _ = _factor(gpu, A, 128, 1, prec=1)
    L, U = oracle.unpack(LU)
    A32 = A.astype(np.float32).astype(np.float64)
    r = np.linalg.norm(A32[oracle.perm_from_ipiv(ipiv)] - L @ U) / (np.linalg.norm(A32) * n * 2.0 ** -24)
    assert r <= 16.0


def test_8192_lookahead_and_solve(gpu):
    import torch
    n = 8192
    A = synth.uniform(n, seed=1)
    b = synth.rhs(n, seed=1)
    for sched in ((128, 1, 16, -1), (256, 1, 16, -1), (256, 2, 32, 1)):
        dA = gpu.to_device(A)
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        assert gpu.lu_factor_ex(dA, ipiv, sched=sched) == 0
        torch.cuda.synchronize()
        assert gpu.lu_factor_info() == (0, 0)
        # scaled factor residual with a library GEMM (rocBLAS via torch) on the device
        L = torch.tril(dA, -1) + torch.eye(n, dtype=torch.float64, device="cuda")
        U = torch.triu(dA)
        perm = torch.tensor(oracle.perm_from_ipiv(ipiv.cpu().numpy()), device="cuda")
        dA0 = gpu.to_device(A)
        R = dA0[perm, :] - L @ U
        rf = (torch.linalg.norm(R) / (torch.linalg.norm(dA0) * n * 2.0 ** -53)).item()
        assert rf <= 16.0, rf
        del L, U, R, dA0
        db = gpu.to_device(b)
        assert gpu.lu_solve_ex(dA, ipiv, db) == 0
        torch.cuda.synchronize()
        x = gpu.to_host(db)[:, 0]
        assert oracle.r_hpl(A, x, b[:, 0]) <= 16.0


def _device_residual(gpu, dA0, dLU, ipiv):
    """||P A - L U||_F / (||A||_F n eps) on the device (tests/residuals.py)."""
    return residuals.factor_residual(dA0, dLU, ipiv)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("b,depth,cus,taper", [(256, 1, 16, -1), (512, 2, 8, -1), (256, 2, 32, 1)])
def test_uniform_32768_schedules(gpu, b, depth, cus, taper):
    """Full-size FP64 look-ahead LU: scaled residual with a library GEMM, the
    pivots are a legal permutation, every multiplier is bounded by 1, the
    first pivot is the plain column search over A, and the whole pivot
    sequence equals the oracle's (tests/golden/xo_uniform_n32768_s1.json holds
    the SHA-256 of the oracle's 32768 pivots for this seeded matrix; rounding
    differences could only change a pivot at a near-tie, which this matrix
    does not have)."""
    import hashlib
    import json
    import torch
    from tests.golden import make_xo
    n = 32768
    with open(make_xo.paths("uniform", n, 1)[1]) as f:
        meta = json.load(f)
    A = synth.uniform(n, seed=1)
    assert make_xo.check_fingerprint(A, meta["fingerprint"]), "regenerated matrix differs"
    dA0 = gpu.to_device(A)
    a00 = A[:, 0].copy()
    del A
    dA = dA0.clone()
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert gpu.lu_factor_ex(dA, ipiv, sched=(b, depth, cus, taper)) == 0
    torch.cuda.synchronize()
    assert gpu.lu_factor_info() == (0, 0)
    ip = ipiv.cpu().numpy()
    assert (ip >= np.arange(n)).all() and (ip < n).all()
    assert ip[0] == int(np.argmax(np.abs(a00)))
    assert hashlib.sha256(ip.astype(np.int32).tobytes()).hexdigest() == meta["ipiv_sha256"]
    assert torch.tril(dA, -1).abs().max().item() <= 1.0
    rf = _device_residual(gpu, dA0, dA, ip)
    assert rf <= 16.0, rf


@pytest.mark.timeout(900)
def test_uniform_40000_per_step_left_swaps(gpu):
    """Past 32768 rows per column segment the left interchanges run as one
    LSWAP task per step instead of the deferred permutation, and panels taller
    than 32768 rows use 1024 rows per work-group: n = 40000 with the tapered
    b = 256 schedule at depth 2 (ragged last panel).  The factorization is
    checked by its scaled residual, legal pivots, bounded multipliers and the
    first pivot, and against the conventional loop (depth 0) of the same
    block size: the same factors and pivots bit for bit, since the look-ahead
    reorders operations only."""
    import torch
    n = 40000
    A = synth.uniform(n, seed=5)
    dA0 = gpu.to_device(A)
    a00 = A[:, 0].copy()
    del A
    results = []
    for depth in (2, 0):
        dA = dA0.clone()
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        print("n=40000 depth %d" % depth, flush=True)
        assert gpu.lu_factor_ex(dA, ipiv, sched=(256, depth, 32, 1)) == 0
        torch.cuda.synchronize()
        assert gpu.lu_factor_info() == (0, 0)
        results.append((dA, ipiv.cpu().numpy()))
    (dA, ip), (dB, ipb) = results
    assert np.array_equal(ip, ipb)
    assert torch.equal(dA, dB)
    del dB
    assert (ip >= np.arange(n)).all() and (ip < n).all()
    assert ip[0] == int(np.argmax(np.abs(a00)))
    assert torch.tril(dA, -1).abs().max().item() <= 1.0
    rf = _device_residual(gpu, dA0, dA, ip)
    assert rf <= 16.0, rf


@pytest.mark.timeout(900)
def test_planted_factors_32768(gpu):
    """A = P L U with L scaled to a = 0.1 sqrt(1024/n) (||L^-1|| as at n=1024):
    the pivots and both factors are recovered."""
    import torch
    n = 32768
    a_l = 0.1 * (1024.0 / n) ** 0.5

    def mm(X, Y):
        return (torch.from_numpy(X).cuda() @ torch.from_numpy(Y).cuda()).cpu().numpy()

    A, L, U, perm = synth.planted(n, seed=4, a_l=a_l, matmul=mm)
    dA = gpu.to_device(A)
    del A
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert gpu.lu_factor_ex(dA, ipiv, sched=(256, 1, 16)) == 0
    torch.cuda.synchronize()
    assert np.array_equal(ipiv.cpu().numpy(), pins.planted_ipiv(perm))
    dL = torch.from_numpy(L).cuda()
    errL = (torch.tril(dA, -1) - torch.tril(dL, -1)).abs().max().item()
    del dL
    dU = torch.from_numpy(U).cuda()
    errU = (torch.triu(dA) - dU).abs().max().item() / dU.abs().max().item()
    assert errL <= 1e-12 and errU <= 1e-12, (errL, errU)
