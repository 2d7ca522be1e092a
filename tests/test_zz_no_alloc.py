"""lu_solve_noalloc (scratch in a static device array, no allocation) against
lu_solve_ex (library-allocated scratch): the same kernels, so the solutions
must agree bit for bit.  Two calls in a row, the second on a smaller system,
so stale ready flags or interchange lists of the first call would show."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _factor(gpu, n, seed, ld):
    import torch
    A = synth.uniform(n, seed=seed)
    dLU = gpu.to_device(A, lda=ld)
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert gpu.lu_factor_ex(dLU, ipiv, prec=gpu.LU_FP64, sched=(64, 1, 16)) == 0
    torch.cuda.synchronize()
    return A, dLU, ipiv


def _rhs(gpu, n, nrhs, seed, ld):
    B = synth.rhs(n, seed=seed, nrhs=nrhs)
    return B, gpu.to_device(B, lda=ld)


@pytest.mark.parametrize("sizes", [((1100, 3, 1131), (333, 2, 333)), ((4096, 1, 4096), (77, 5, 80))])
def test_noalloc_matches_solve_ex(gpu, sizes):
    import torch
    for call, (n, nrhs, ld) in enumerate(sizes):
        print("noalloc call %d: n=%d nrhs=%d ld=%d" % (call, n, nrhs, ld), flush=True)
        A, dLU, ipiv = _factor(gpu, n, seed=10 + call, ld=ld)
        B, dB1 = _rhs(gpu, n, nrhs, seed=20 + call, ld=ld)
        _, dB2 = _rhs(gpu, n, nrhs, seed=20 + call, ld=ld)
        assert gpu.lu_solve_ex(dLU, ipiv, dB1) == 0
        assert gpu.lu_solve_noalloc(dLU, ipiv, dB2) == 0
        torch.cuda.synchronize()
        X1 = gpu.to_host(dB1)
        X2 = gpu.to_host(dB2)
        assert np.array_equal(X1.view(np.uint64), X2.view(np.uint64)), \
            "max diff %g" % np.abs(X1 - X2).max()
        for c in range(nrhs):
            assert oracle.r_hpl(A, X2[:, c], B[:, c]) <= 16.0


def test_noalloc_rejects_oversize(gpu):
    import torch
    n = gpu.LU_NOALLOC_MAX_N + 1
    small = torch.zeros(4, dtype=torch.float64, device="cuda")
    piv = torch.zeros(4, dtype=torch.int32, device="cuda")
    lib = gpu.load()
    rc = lib.lu_solve_noalloc(n, 1, small.data_ptr(), n, piv.data_ptr(), small.data_ptr(), n, None)
    assert rc == gpu.LU_ERR_UNSUPPORTED
    assert lib.lu_solve_noalloc(0, 1, 0, 1, 0, 0, 1, None) == 0
    assert lib.lu_solve_noalloc(5, 1, small.data_ptr(), 4, piv.data_ptr(), small.data_ptr(), 5, None) == -4
