"""Per-kernel parity on the GPU: each step of one LU iteration against the
oracle or an exact/bounded CPU reference (numpy FP64), through the C ABI."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_mfma_f64_lane_layout(gpu):
    """Pins the result layout the FP64 GEMM relies on: lane l, register r of
    v_mfma_f64_16x16x4f64 holds D[l/16 + 4r][l%16] (A lane l = (i=l%16, k=l/16),
    B lane l = (k=l/16, j=l%16))."""
    import torch
    out = torch.zeros(256, dtype=torch.float64, device="cuda")
    assert gpu.lu_k_probe_mfma_f64(out) == 0
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(64, 4)
    for lane in range(64):
        for r in range(4):
            i, j = lane // 16 + 4 * r, lane % 16
            want = sum((i + 16 * k) * (100.0 + j + 16 * k) for k in range(4))
            assert got[lane, r] == want, (lane, r)


def _gemm_case(gpu, prec, m, n, k, seed):
    import torch
    g = np.random.default_rng(seed)
    A = np.asfortranarray(g.uniform(-1, 1, (m, k)))
    B = np.asfortranarray(g.uniform(-1, 1, (k, n)))
    C = np.asfortranarray(g.uniform(-1, 1, (m, n)))
    dt = torch.float64 if prec == gpu.LU_FP64 else torch.float32
    dA, dB, dC = gpu.to_device(A, dt), gpu.to_device(B, dt), gpu.to_device(C, dt, lda=m + 3)
    assert gpu.lu_k_gemm(dA, dB, dC, prec=prec) == 0
    torch.cuda.synchronize()
    return A, B, C, gpu.to_host(dC).astype(np.float64)


@pytest.mark.parametrize("m,n,k", [(128, 128, 16), (130, 70, 16), (300, 257, 64), (256, 512, 256),
                                   (77, 200, 100), (1, 1, 1), (513, 129, 512)])
def test_gemm_f64(gpu, m, n, k):
    A, B, C, got = _gemm_case(gpu, gpu.LU_FP64, m, n, k, m + n + k)
    want = C - A @ B
    # FP64 error bound of a k-term dot product: k * 2^-53 * sum |a||b| (+ the subtraction)
    bound = (k + 2) * 2.0 ** -53 * (np.abs(A) @ np.abs(B) + np.abs(C))
    assert (np.abs(got - want) <= bound).all()


@pytest.mark.parametrize("m,n,k", [(130, 70, 16), (300, 257, 64), (256, 512, 256)])
def test_gemm_f32(gpu, m, n, k):
    A, B, C, got = _gemm_case(gpu, gpu.LU_FP32, m, n, k, 7 + m)
    A32, B32, C32 = (x.astype(np.float32).astype(np.float64) for x in (A, B, C))
    want = C32 - A32 @ B32
    bound = (k + 2) * 2.0 ** -24 * (np.abs(A32) @ np.abs(B32) + np.abs(C32))
    assert (np.abs(got - want) <= bound).all()


@pytest.mark.parametrize("prec,u", [(2, 2.0 ** -11), (3, 2.0 ** -8)])
@pytest.mark.parametrize("m,n,k", [(130, 70, 32), (300, 257, 256), (64, 64, 100)])
def test_gemm_half_precision_operands(gpu, prec, u, m, n, k):
    A, B, C, got = _gemm_case(gpu, prec, m, n, k, 11 + k)
    A32, B32, C32 = (x.astype(np.float32).astype(np.float64) for x in (A, B, C))
    want = C32 - A32 @ B32
    # each operand rounded once to the half format (relative u), FP32 accumulation
    bound = (2 * u + (k + 2) * 2.0 ** -24) * (np.abs(A32) @ np.abs(B32)) + 2.0 ** -23 * np.abs(C32)
    assert (np.abs(got - want) <= bound).all()


def _square_with_panel(m, w, seed):
    A = synth.uniform(m, seed=seed)
    return np.array(A, order="F"), w


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("m,w,wgs", [(64, 64, 1), (700, 16, 4), (1000, 64, 8), (1000, 100, 3),
                                     (2500, 256, 16), (300, 33, 2), (4096, 512, 8),
                                     (1000, 128, 1), (512, 256, 1), (257, 33, 1), (1024, 512, 1)])
def test_panel_matches_oracle(gpu, prec, m, w, wgs):
    import torch
    A, _ = _square_with_panel(m, w, seed=m + w)
    LU, ipiv, _ = oracle.getrf(A, nthreads=8)
    dt = torch.float64 if prec == 0 else torch.float32
    P = gpu.to_device(A[:, :w], dt, lda=m + 5)
    piv = torch.zeros(w, dtype=torch.int32, device="cuda")
    assert gpu.lu_k_panel(P, piv, prec=prec, wgs=wgs) == 0
    torch.cuda.synchronize()
    got = gpu.to_host(P).astype(np.float64)
    gp = piv.cpu().numpy()
    if prec == 0:
        assert np.array_equal(gp, ipiv[:w])
        # the oracle factored the whole matrix: its later interchanges (steps >= w)
        # also moved rows of the first w columns; apply them to the panel result
        for t in range(w, m):
            if ipiv[t] != t:
                got[[t, ipiv[t]], :] = got[[ipiv[t], t], :]
        assert np.abs(got - LU[:, :w]).max() <= 1e-12 * max(1.0, np.abs(LU[:, :w]).max())
    else:
        # FP32 panel: compare the factorization property of the panel itself
        perm = np.arange(m)
        for t in range(w):
            perm[[t, gp[t]]] = perm[[gp[t], t]]
        L = np.tril(got, -1)[:, :w] + np.eye(m, w)
        U = np.triu(got[:w, :w])
        PA = A[perm, :w].astype(np.float32).astype(np.float64)
        err = np.abs(PA - L @ U).max()
        assert err <= 4 * w * 2.0 ** -24 * np.abs(L).max() * np.abs(U).max() * 4
        assert np.abs(np.tril(got, -1)).max() <= 1.0


@pytest.mark.parametrize("m,w,ncols", [(200, 64, 50), (1000, 128, 300), (600, 256, 257)])
def test_update_matches_numpy(gpu, m, w, ncols):
    import torch
    A = synth.uniform(m, seed=w)
    LU, ipiv, _ = oracle.getrf(A)           # factored panel = first w columns
    g = np.random.default_rng(ncols)
    C = g.uniform(-1, 1, (m, ncols))
    M = np.asfortranarray(np.hstack([LU[:, :w], C]))
    dM = gpu.to_device(M)
    piv = torch.tensor(ipiv[:w], dtype=torch.int32, device="cuda")
    assert gpu.lu_k_update(dM[:, :w], piv, dM[:, w:]) == 0
    torch.cuda.synchronize()
    got = gpu.to_host(dM)[:, w:]
    want = C.copy()
    for t in range(w):
        want[[t, ipiv[t]], :] = want[[ipiv[t], t], :]
    L11 = np.tril(LU[:w, :w], -1) + np.eye(w)
    want[:w] = sla.solve_triangular(L11, want[:w], lower=True, unit_diagonal=True)
    want[w:] -= LU[w:, :w] @ want[:w]
    assert np.abs(got - want).max() <= 1e-11 * max(1.0, np.abs(want).max())


@pytest.mark.parametrize("m,w", [(100, 32), (3000, 512), (513, 512)])
def test_laswp_exact(gpu, m, w):
    import torch
    g = np.random.default_rng(m)
    piv = np.array([t + g.integers(0, m - t) for t in range(w)], dtype=np.int32)
    C = g.uniform(-1, 1, (m, 37))
    dC = gpu.to_device(C)
    dp = torch.tensor(piv, device="cuda")
    assert gpu.lu_k_laswp(dC, dp, w) == 0
    torch.cuda.synchronize()
    want = C.copy()
    for t in range(w):
        want[[t, piv[t]], :] = want[[piv[t], t], :]
    assert np.array_equal(gpu.to_host(dC), want)


WIDE_CHILD = r"""
import sys
sys.path.insert(0, %r)
import numpy as np
import torch
import paper_1804_07017_amd as lu
import synth
lu.load()
m, w, out = %d, %d, %r
A = synth.uniform(m, seed=m + w)
P = lu.to_device(np.array(A[:, :w], order="F"), torch.float64, lda=m + 5)
piv = torch.zeros(w, dtype=torch.int32, device="cuda")
print("case wide panel m=%%d w=%%d" %% (m, w), flush=True)
rc = lu.lu_k_panel(P, piv, prec=0, wgs=1)
torch.cuda.synchronize()
np.save(out + "/lu.npy", lu.to_host(P))
np.save(out + "/piv.npy", piv.cpu().numpy())
print("rc", rc, flush=True)
"""


@pytest.mark.parametrize("m,w", [(4096, 256), (3000, 200)])
def test_wide_fp64_panel_matches_oracle(gpu, tmp_path, m, w):
    """The FP64 panel variant for tall panels (1024 rows per work-group, its
    finished columns re-read from memory instead of an LDS copy), which
    factors the panels taller than LU_WIDE_ROWS rows (20480 by default).  A
    child process lowers that threshold to 512 rows so the variant runs at a
    size the oracle finishes quickly; the result is compared element by
    element, as for the other panel variants."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, LU_WIDE_ROWS="512")
    r = subprocess.run([sys.executable, "-c", WIDE_CHILD % (root, m, w, str(tmp_path))], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "rc 0" in r.stdout, (r.stdout[-2000:], r.stderr[-2000:])
    got = np.load(str(tmp_path / "lu.npy"))
    gp = np.load(str(tmp_path / "piv.npy"))
    A = synth.uniform(m, seed=m + w)
    LU, ipiv, _ = oracle.getrf(A, nthreads=8)
    assert np.array_equal(gp, ipiv[:w])
    for t in range(w, m):
        if ipiv[t] != t:
            got[[t, ipiv[t]], :] = got[[ipiv[t], t], :]
    assert np.abs(got - LU[:, :w]).max() <= 1e-12 * max(1.0, np.abs(LU[:, :w]).max())


def test_xcd_probe_round_robin(gpu):
    """The XCD-island schedule keeps the panels on XCD 0 by relying on the
    round-robin deal of work-groups to the 8 XCDs (work-group b on XCD
    (b + c) % 8 for an offset c of the launch).  The probe reads the XCC_ID
    register of 64 work-groups; the library's verdict must match what it
    read, and on an MI355X in its single-partition mode the deal holds."""
    import numpy as np
    import torch
    out = np.full(64, -1, dtype=np.int32)
    rc = gpu.load().lu_k_xcd_probe(out.ctypes.data)
    assert rc in (0, 1), rc
    assert np.all((out >= 0) & (out < 8))
    rr = bool(np.all((out - out[0] - np.arange(64)) % 8 == 0))
    assert rc == int(rr), out.tolist()
    if torch.cuda.get_device_properties(0).multi_processor_count == 256:
        assert rr, out.tolist()
