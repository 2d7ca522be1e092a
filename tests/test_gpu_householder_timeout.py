"""The panel-barrier time-out path of the Householder entry points, forced from
the host: a child process sets the library's wall-clock bound on a barrier
wait to one tick (LU_DEBUG_BARRIER_SPIN, read when the library first touches
the device), so the panel kernel's bounded waits end early and every kernel
still exits normally.  QR and the band reduction carry no index arrays, so a
panel that gives up leaves wrong values but no out-of-range access.  Each
call must still enqueue (0) and lu_factor_info must report LU_ERR_BARRIER,
again for a repeated call (the error words are reset after each report and
every later wait ends at the same bound)."""
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
g.manual_seed(2)
A = lu.colmajor(n)
A.uniform_(-1.0, 1.0, generator=g)
tau = torch.zeros(n, dtype=torch.float64, device="cuda")
torch.cuda.synchronize()
print("qr", lu.qr_factor(A, tau), lu.lu_factor_info()[0], flush=True)
print("qr-again", lu.qr_factor(A, tau), lu.lu_factor_info()[0], flush=True)
A.uniform_(-1.0, 1.0, generator=g)
tq = torch.zeros(n, dtype=torch.float64, device="cuda")
tp = torch.zeros(n, dtype=torch.float64, device="cuda")
torch.cuda.synchronize()
print("band", lu.band_reduce(A, 128, tq, tp), lu.lu_factor_info()[0], flush=True)
"""


def test_barrier_timeout_reported():
    import paper_1804_07017_amd as lu
    env = dict(os.environ, LU_DEBUG_BARRIER_SPIN="1")
    r = subprocess.run([sys.executable, "-c", CHILD % ROOT], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    rows = {line.split()[0]: [int(x) for x in line.split()[1:]] for line in r.stdout.splitlines() if line.strip()}
    # enqueue succeeds; the status of the factorization is the barrier time-out
    assert rows["qr"] == [0, lu.LU_ERR_BARRIER], r.stdout
    assert rows["qr-again"] == [0, lu.LU_ERR_BARRIER], r.stdout
    assert rows["band"] == [0, lu.LU_ERR_BARRIER], r.stdout
