"""The LU entry points under a panel-barrier time-out, forced from the host:
a child process sets the library's wall-clock bound on a barrier wait to one
tick (LU_DEBUG_BARRIER_SPIN, read when the library first touches the device),
so every multi-work-group panel gives up at its first wait and every kernel
still exits normally.  A panel that gives up leaves an empty interchange list
(written at its start) and the trailing kernels read lists defensively, so
the factorization finishes with wrong values but no out-of-range access:
lu_factor_ex enqueues (0), lu_factor_info reports LU_ERR_BARRIER (again on a
repeated call), and lu_solve_ir reports LU_ERR_BARRIER instead of a solution.
The child prints the case before each step so that a failure names it."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, %r)
import torch
import paper_1804_07017_amd as lu
lu.load()
n = 4096
g = torch.Generator(device="cuda")
g.manual_seed(3)
A = lu.colmajor(n)
A.uniform_(-1.0, 1.0, generator=g)
A0 = A.clone()
ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
torch.cuda.synchronize()
for case, prec in (("fp64", lu.LU_FP64), ("fp64-again", lu.LU_FP64)):
    A.copy_(A0)
    print("case", case, flush=True)
    rc = lu.lu_factor_ex(A, ipiv, prec=prec, sched=(256, 2, 32))
    print(case, rc, lu.lu_factor_info()[0], flush=True)
A32 = A0.to(torch.float32)
print("case fp32", flush=True)
rc = lu.lu_factor_ex(A32, ipiv, prec=lu.LU_FP32, sched=(256, 1, 16))
print("fp32", rc, lu.lu_factor_info()[0], flush=True)
b = torch.ones(n, dtype=torch.float64, device="cuda")
x = torch.zeros(n, dtype=torch.float64, device="cuda")
print("case ir", flush=True)
st, it, res = lu.lu_solve_ir(A0, b, x, prec=lu.LU_MIXED_FP16, max_iter=5)
print("ir", st, 0, flush=True)
"""


def test_lu_barrier_timeout_reported():
    import paper_1804_07017_amd as lu
    env = dict(os.environ, LU_DEBUG_BARRIER_SPIN="1")
    r = subprocess.run([sys.executable, "-c", CHILD % ROOT], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    rows = {line.split()[0]: [int(x) for x in line.split()[1:]] for line in r.stdout.splitlines()
            if line.strip() and not line.startswith("case")}
    assert rows["fp64"] == [0, lu.LU_ERR_BARRIER], r.stdout
    assert rows["fp64-again"] == [0, lu.LU_ERR_BARRIER], r.stdout
    assert rows["fp32"] == [0, lu.LU_ERR_BARRIER], r.stdout
    assert rows["ir"] == [lu.LU_ERR_BARRIER, 0], r.stdout
