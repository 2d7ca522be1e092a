"""Write the FP64 oracle solutions x_o of the n = 32768 refinement workloads.

The mixed-precision path is judged by the error of its refined solution
against the plain FP64 solution x_o = getrs(getrf(A), b) of the CPU oracle
(unblocked Gaussian elimination with partial pivoting, the decomposition of
Sec. 3.4 / operations RL1-RL3 of Sec. 3.5).  At n = 32768 the oracle takes an
hour or more on a few cores, so its solution is computed once per workload by
this script and stored next to it:

  xo_<workload>_n<n>_s<seed>.npy    x_o (float64[n])
  xo_<workload>_n<n>_s<seed>.json   the oracle's ipiv digest, INFO, wall time,
                                    the HPL residual of x_o and a fingerprint
                                    of A (trace and sampled entries) that
                                    readers check before using x_o

Workloads: ``dominant`` (uniform[-1,1) with a_ii = the row's absolute sum) and
``uniform`` (i.i.d. uniform[-1,1)), right-hand side ``synth.rhs(n, seed)``.
Only ``synth`` (the seeded generators) and ``oracle`` are used.

usage: python tests/golden/make_xo.py {dominant|uniform} [n] [seed] [threads] [outdir]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

FINGERPRINT_SAMPLES = 4096


def fingerprint(A: np.ndarray, seed: int = 12345) -> dict:
    """Trace and a seeded sample of entries: enough to tell whether a
    regenerated matrix is the one x_o was computed for."""
    n = A.shape[0]
    g = np.random.Generator(np.random.Philox(key=[seed, 99]))
    i = g.integers(0, n, FINGERPRINT_SAMPLES)
    j = g.integers(0, n, FINGERPRINT_SAMPLES)
    vals = np.ascontiguousarray(A[i, j])
    return {"trace": float(np.trace(A)), "rows": i.tolist(), "cols": j.tolist(),
            "sha256_samples": hashlib.sha256(vals.tobytes()).hexdigest()}


def check_fingerprint(A: np.ndarray, fp: dict) -> bool:
    i = np.asarray(fp["rows"])
    j = np.asarray(fp["cols"])
    vals = np.ascontiguousarray(A[i, j])
    return hashlib.sha256(vals.tobytes()).hexdigest() == fp["sha256_samples"] and \
        float(np.trace(A)) == fp["trace"]


def paths(workload: str, n: int, seed: int, outdir: str | None = None):
    d = outdir or os.path.dirname(os.path.abspath(__file__))
    stem = os.path.join(d, "xo_%s_n%d_s%d" % (workload, n, seed))
    return stem + ".npy", stem + ".json"


def make_matrix(workload: str, n: int, seed: int) -> np.ndarray:
    if workload == "dominant":
        return synth.dominant(n, seed)
    if workload == "uniform":
        return synth.uniform(n, seed)
    raise ValueError("unknown workload %r" % workload)


def main(argv) -> int:
    workload = argv[1]
    n = int(argv[2]) if len(argv) > 2 else 32768
    seed = int(argv[3]) if len(argv) > 3 else 1
    threads = int(argv[4]) if len(argv) > 4 else (os.cpu_count() or 1)
    outdir = argv[5] if len(argv) > 5 else None
    t0 = time.time()
    A = make_matrix(workload, n, seed)
    b = synth.rhs(n, seed)[:, 0].copy()
    fp = fingerprint(A)
    print("make_xo: %s n=%d seed=%d generated in %.1f s" % (workload, n, seed, time.time() - t0), flush=True)
    t1 = time.time()
    LU, ipiv, info = oracle.getrf(A, nthreads=threads)
    t_f = time.time() - t1
    print("make_xo: oracle getrf %.1f s (%d threads), info %d" % (t_f, threads, info), flush=True)
    if info != 0:
        raise SystemExit("singular matrix, info %d" % info)
    x = oracle.getrs(LU, ipiv, b)
    del LU
    res = oracle.r_hpl(A, x, b)
    swaps = int(np.count_nonzero(ipiv != np.arange(n)))
    npy, js = paths(workload, n, seed, outdir)
    np.save(npy, x)
    meta = {"workload": workload, "n": n, "seed": seed, "rhs": "synth.rhs(n, seed)[:, 0]",
            "oracle_threads": threads, "oracle_getrf_s": round(t_f, 1), "info": int(info),
            "interchanges": swaps, "ipiv_sha256": hashlib.sha256(ipiv.astype(np.int32).tobytes()).hexdigest(),
            "hpl_resid_xo": res, "x_inf": float(np.abs(x).max()), "fingerprint": fp}
    with open(js, "w") as f:
        json.dump(meta, f)
    print("make_xo: wrote %s (R_hpl %.4f, %d interchanges)" % (npy, res, swaps), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
