"""Host-side pieces of bench.py that need no GPU: the CPU oracle rates and
the LU baseline return the documented fields on a tiny budget, and
--gpus N > 1 exits with a message before anything touches a device."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("kind", ["chol", "qr", "band"])
def test_oracle_rate_fields(kind):
    r = bench.oracle_rate(kind, budget_s=0.05)
    assert r["kind"] == "oracle" and r["unit"] == "GFLOP/s" and r["value"] > 0
    assert r["cores"] >= 1 and "matrix" in r["sample"]
    json.dumps(r)


def test_cpu_baseline_fields():
    r = bench.cpu_baseline(budget_s=0.05)
    assert r["kind"] == "oracle" and r["value"] > 0 and r["cores"] >= 1
    # every core of the affinity mask, and the host described
    assert r["cores"] == len(os.sched_getaffinity(0)) == r["affinity"]
    assert r["nproc"] >= r["affinity"] and r["cpu_model"]
    json.dumps(r)


def test_oracle_solution_fingerprint():
    """The bench compares the refined n = 32768 solution with the oracle's
    stored one only after checking that the regenerated row-dominant matrix
    is the one the oracle solved (here at a small size: the fingerprint of a
    matrix matches itself and not a perturbed copy)."""
    import synth
    from tests.golden import make_xo
    A = synth.dominant(300, seed=1)
    fp = make_xo.fingerprint(A)
    assert bench.same_matrix(A, fp)
    B = A.copy()
    i, j = fp["rows"][7], fp["cols"][7]
    B[i, j] += 1e-13
    assert not bench.same_matrix(B, fp)
    assert bench.oracle_solution(300) == (None, None)


def test_several_gpus_exit_with_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr and not p.stdout.strip()
