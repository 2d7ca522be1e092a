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
    json.dumps(r)


def test_several_gpus_exit_with_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr and not p.stdout.strip()
