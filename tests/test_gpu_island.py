"""The XCD-island schedule (opt-in, LU_ISLAND=1): with look-ahead every panel
runs on XCD 0 and the kernels of the update stream leave XCD 0 free, claiming
their tiles, slabs or column blocks from counters.  Each element still sees
the same operations in the same order, so a child process with the island on
must reproduce, bit for bit, the factors of the default schedule (computed in
this process), which in turn match the oracle (test_gpu_factor.py).  The
child prints the case before each step so that a failure names it."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, %r)
import numpy as np
import torch
import paper_1804_07017_amd as lu
import synth
lu.load()
out = %r
for n, b, depth, prec in ((1500, 128, 1, 0), (2100, 256, 2, 0), (2100, 128, 2, 2)):
    print("case", n, b, depth, prec, flush=True)
    A = synth.uniform(n, seed=n + b)
    dt = torch.float64 if prec == 0 else torch.float32
    dA = lu.to_device(A, dt)
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    rc = lu.lu_factor_ex(dA, ipiv, prec=prec, sched=(b, depth, 16))
    rc2, info = lu.lu_factor_info()
    torch.cuda.synchronize()
    np.save(out + "/lu_%%d_%%d_%%d_%%d.npy" %% (n, b, depth, prec), lu.to_host(dA))
    np.save(out + "/ip_%%d_%%d_%%d_%%d.npy" %% (n, b, depth, prec), ipiv.cpu().numpy())
    print("done", rc, rc2, info, flush=True)
"""


def test_island_schedule_bitwise_equal_to_default(gpu, tmp_path):
    import torch
    env = dict(os.environ, LU_ISLAND="1")
    r = subprocess.run([sys.executable, "-c", CHILD % (ROOT, str(tmp_path))], env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert r.stdout.count("done 0 0 0") == 3, r.stdout
    for n, b, depth, prec in ((1500, 128, 1, 0), (2100, 256, 2, 0), (2100, 128, 2, 2)):
        A = synth.uniform(n, seed=n + b)
        dt = torch.float64 if prec == 0 else torch.float32
        dA = gpu.to_device(A, dt)
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        assert gpu.lu_factor_ex(dA, ipiv, prec=prec, sched=(b, depth, 16)) == 0
        torch.cuda.synchronize()
        got = np.load(str(tmp_path / ("lu_%d_%d_%d_%d.npy" % (n, b, depth, prec))))
        gip = np.load(str(tmp_path / ("ip_%d_%d_%d_%d.npy" % (n, b, depth, prec))))
        assert np.array_equal(gip, ipiv.cpu().numpy())
        assert np.array_equal(got.view(np.int64) if got.dtype == np.float64 else got.view(np.int32),
                              gpu.to_host(dA).view(np.int64) if prec == 0 else gpu.to_host(dA).view(np.int32))
        if prec == 0:
            assert oracle.r_factor(A, got, gip) <= 16.0
