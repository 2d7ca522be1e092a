"""Benchmark: look-ahead LU at n = 32768 on one MI355X.

One step = the whole hot path on one batch of synthetic input resident in HBM:
  1. FP64 look-ahead LU (lu_factor) of a uniform[-1,1) n x n matrix
     (restored from a pristine device copy first; the copy is outside the
     factorization's event timing),
  2. lu_solve with one uniform[-1,1) right-hand side,
  3. lu_solve_ir in mixed precision (FP16 trailing GEMM, FP32 panel/TRSM, FP64
     refinement) on the row-dominant matrix of the same size.
`value` is the FP64 factorization rate 2/3 n^3 / t_factor (median over the
timed steps, HIP events on the stream the factorization runs on).  The
row-dominant matrix and its right-hand side come from the seeded host
generators (synth), so that the refined solution can be compared with the
oracle's FP64 solution stored in tests/golden (when one exists for n).
After the timed steps, untimed for the headline: one FP64 and one mixed
factorization with the library's per-launch GEMM timing hook (the rooflines),
optionally the standalone GEMM ceiling (--gemm-ceiling), the Cholesky, QR and
band-reduction legs (each timed like the LU), then the CPU oracles on bounded
samples.

Prints one JSON line.  --gpus N with N > 1 exits: the path runs on one GPU.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LU GFLOPS (2/3·n³/t) at n=32768, FP64 vs mixed+IR; % MFMA peak; IR time-to-solve"
FP64_PEAK_TFLOPS = 78.6
FP16_PEAK_TFLOPS = 2516.6     # dense FP16/BF16 matrix peak
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the FP64 trailing GEMM, from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE) over one bench step, each scaled by what the same
# counter reads for the bench's own n*n*8-byte device copy (see
# profiles/gemm_f64_n32768_hbm_traffic.md).  Valid only for the schedule and the
# GEMM source it was measured with; otherwise the bench reports null.
GEMM_TRAFFIC = {"n": 32768, "b": 256, "depth": 2, "taper": 1, "gemm_source_sha256_16": "43f530c178969ad6",
                "bytes_per_launch": 2098771685}


def gemm_source_hash():
    import hashlib
    path = os.path.join(ROOT, "paper_1804_07017_amd", "csrc", "gemm.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def gemm_algorithmic_bytes(lu, n, b, depth, taper):
    """Mean per-launch bytes the trailing GEMMs of one factorization must move:
    C read and written once, A21 and U12 read once (8-byte elements)."""
    rc, starts = lu.lu_plan_panels(n, b, taper, lu.LU_FP64)
    rc, tasks = lu.lu_plan_build_panels(n, starts, depth)
    tot, cnt = 0.0, 0
    for t in tasks:
        if t["kind"] != lu.LU_TASK_UPDATE:
            continue
        kb = starts[t["step"]]
        wk = starts[t["step"] + 1] - kb
        m, w = n - kb - wk, t["col_end"] - t["col_begin"]
        if m > 0 and w > 0:
            tot += 16.0 * m * w + 8.0 * m * wk + 8.0 * wk * w
            cnt += 1
    return tot / max(cnt, 1)


def oracle_solution(n, workload="dominant", seed=1):
    """The oracle's FP64 solution of the seeded system of size n (workload
    "dominant" or "uniform"), as written by tests/golden/make_xo.py
    (float64[n]), with its metadata, or (None, None) when none is stored for n."""
    import numpy as np
    stem = os.path.join(ROOT, "tests", "golden", "xo_%s_n%d_s%d" % (workload, n, seed))
    if not (os.path.exists(stem + ".npy") and os.path.exists(stem + ".json")):
        return None, None
    with open(stem + ".json") as f:
        meta = json.load(f)
    return np.load(stem + ".npy"), meta


def same_matrix(A, fp):
    """Does the host matrix A carry the fingerprint (trace and a hash of
    sampled entries) recorded with the oracle's solution?"""
    import hashlib
    import numpy as np
    i = np.asarray(fp["rows"])
    j = np.asarray(fp["cols"])
    vals = np.ascontiguousarray(A[i, j])
    return hashlib.sha256(vals.tobytes()).hexdigest() == fp["sha256_samples"] and float(np.trace(A)) == fp["trace"]


def cpu_info():
    """Host CPU facts for the baseline: online CPUs, the process's affinity
    mask size and the CPU model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model}


def device_spd(lu, n, seed, A):
    """SPD workload on the device, written into the column-major n x n tensor
    A: the symmetric part (B + B^T)/2 of a uniform[-1,1) matrix B with each
    diagonal entry set to its row's absolute sum (strictly diagonally
    dominant).  Temporaries stay at 4096-column blocks."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    A.uniform_(-1.0, 1.0, generator=g)
    for c0 in range(0, n, 4096):
        c1 = min(n, c0 + 4096)
        sym = (A[c0:c1, :].clone() + A[:, c0:c1].t()) / 2.0
        A[c0:c1, :] = sym
        A[:, c0:c1] = sym.t()
        del sym
    rowsum = torch.zeros(n, dtype=A.dtype, device=A.device)
    for c0 in range(0, n, 4096):
        rowsum += A[:, c0:min(n, c0 + 4096)].abs().sum(dim=1)
    A.diagonal().copy_(rowsum)
    return A


def cholesky_leg(lu, n, reps, A0, A):
    """FP64 Cholesky with look-ahead (chol_factor, default schedule) on the SPD
    workload: median over reps timed factorizations after one warm-up, HIP
    events on the factorization's stream; the pristine matrix is restored
    before each run outside the timed region."""
    import torch
    device_spd(lu, n, 7, A0)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()             # the input is built on the default stream
    ts = []
    for r in range(reps + 1):
        with torch.cuda.stream(stream):
            A.copy_(A0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rc = lu.chol_factor(A, stream=stream)
            e1.record(stream)
        stream.synchronize()
        if rc != 0:
            raise RuntimeError("chol_factor returned %d" % rc)
        st, info = lu.lu_factor_info()
        if r:
            ts.append(e0.elapsed_time(e1))
        print("bench: cholesky run %d %.1f ms status %d info %d" % (r, e0.elapsed_time(e1), st, info),
              file=sys.stderr, flush=True)
        if st != 0 or info != 0:
            raise RuntimeError("cholesky: status %d info %d" % (st, info))
    t = statistics.median(ts)
    gf = n ** 3 / 3.0 / (t * 1e-3) / 1e9
    # one right-hand side with the last factor (chol_solve, potrs semantics):
    # median over reps timed solves, each from the same b; HPL residual of the
    # last against the pristine matrix (a device GEMV in FP64)
    g = torch.Generator(device="cuda")
    g.manual_seed(8)
    bvec = torch.empty(n, dtype=torch.float64, device=A.device).uniform_(-1.0, 1.0, generator=g)
    x = torch.empty_like(bvec)
    tss = []
    for r in range(reps + 1):
        with torch.cuda.stream(stream):
            x.copy_(bvec)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rc = lu.chol_solve(A, x, stream=stream)
            e1.record(stream)
        stream.synchronize()
        if rc != 0:
            raise RuntimeError("chol_solve returned %d" % rc)
        if r:
            tss.append(e0.elapsed_time(e1))
    with torch.no_grad():
        a_inf = 0.0
        for c0 in range(0, n, 4096):
            a_inf = max(a_inf, A0[c0:min(n, c0 + 4096), :].abs().sum(dim=1).max().item())
        res = (A0 @ x - bvec).abs().max().item()
        hpl = res / (2.0 ** -53 * (a_inf * x.abs().max().item() + bvec.abs().max().item()) * n)
    return {"workload": "FP64 Cholesky with look-ahead of an SPD n=%d matrix (symmetric uniform[-1,1) part, "
                        "diagonal = row absolute sum)" % n,
            "schedule": {"b": 256, "depth": 2, "panel_cus": 32}, "t_factor_ms": round(t, 3),
            "gflops": round(gf, 1), "flops": "n^3/3", "pct_fp64_peak": round(100 * gf / 1e3 / FP64_PEAK_TFLOPS, 2),
            "t_solve_ms": round(statistics.median(tss), 3), "hpl_resid": hpl, "runs": reps}


def qr_leg(lu, n, reps, A0, A):
    """FP64 Householder QR with look-ahead (qr_factor, default schedule) of a
    uniform[-1,1) n x n matrix: median over reps timed factorizations after one
    warm-up, HIP events on the factorization's stream; the pristine matrix is
    restored before each run outside the timed region.  GFLOP/s counts the
    geqrf flops 2mn^2 - 2n^3/3 = 4n^3/3 at m = n."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    A0.uniform_(-1.0, 1.0, generator=g)
    tau = torch.zeros(n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()             # the input is built on the default stream
    ts = []
    for r in range(reps + 1):
        with torch.cuda.stream(stream):
            A.copy_(A0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rc = lu.qr_factor(A, tau, stream=stream)
            e1.record(stream)
        stream.synchronize()
        if rc != 0:
            raise RuntimeError("qr_factor returned %d" % rc)
        st, _ = lu.lu_factor_info()
        if r:
            ts.append(e0.elapsed_time(e1))
        print("bench: qr run %d %.1f ms status %d" % (r, e0.elapsed_time(e1), st), file=sys.stderr, flush=True)
        if st != 0:
            raise RuntimeError("qr: status %d" % st)
    t = statistics.median(ts)
    gf = 4.0 * n ** 3 / 3.0 / (t * 1e-3) / 1e9
    # |R[0,0]| is the 2-norm of column 0 of A; a cheap sanity check of the run
    r00 = abs(float(A[0, 0]))
    c0 = float(torch.linalg.vector_norm(A0[:, 0]))
    if abs(r00 - c0) > 1e-10 * c0:
        raise RuntimeError("qr: |R[0,0]| = %r, column norm %r" % (r00, c0))
    del tau
    return {"workload": "FP64 Householder QR with look-ahead of a uniform[-1,1) %d x %d matrix" % (n, n),
            "schedule": {"b": 128, "depth": 2}, "t_factor_ms": round(t, 3), "gflops": round(gf, 1),
            "flops": "4n^3/3", "pct_fp64_peak": round(100 * gf / 1e3 / FP64_PEAK_TFLOPS, 2), "runs": reps}


def band_leg(lu, n, w, reps, A0, A):
    """FP64 two-sided reduction to band form (band_reduce, bandwidth w) of a
    uniform[-1,1) n x n matrix: median over reps timed runs after one warm-up,
    HIP events on the reduction's stream; the pristine matrix is restored
    before each run outside the timed region.  GFLOP/s on the 8n^3/3 count of
    the full bidiagonal reduction, as the paper reports it."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(13)
    A0.uniform_(-1.0, 1.0, generator=g)
    tq = torch.zeros(n, dtype=torch.float64, device="cuda")
    tp = torch.zeros(n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()             # the input is built on the default stream
    ts = []
    for r in range(reps + 1):
        with torch.cuda.stream(stream):
            A.copy_(A0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rc = lu.band_reduce(A, w, tq, tp, stream=stream)
            e1.record(stream)
        stream.synchronize()
        if rc != 0:
            raise RuntimeError("band_reduce returned %d" % rc)
        st, _ = lu.lu_factor_info()
        if r:
            ts.append(e0.elapsed_time(e1))
        print("bench: band run %d %.1f ms status %d" % (r, e0.elapsed_time(e1), st), file=sys.stderr, flush=True)
        if st != 0:
            raise RuntimeError("band: status %d" % st)
    t = statistics.median(ts)
    gf = 8.0 * n ** 3 / 3.0 / (t * 1e-3) / 1e9
    # |B[0,0]| is the 2-norm of column 0 of A, and the band keeps ||A||_F
    r00 = abs(float(A[0, 0]))
    c0 = float(torch.linalg.vector_norm(A0[:, 0]))
    if abs(r00 - c0) > 1e-10 * c0:
        raise RuntimeError("band: |B[0,0]| = %r, column norm %r" % (r00, c0))
    del tq, tp
    return {"workload": "FP64 two-sided reduction to upper band form (SVD stage 1) of a uniform[-1,1) "
                        "%d x %d matrix, bandwidth %d" % (n, n, w),
            "w": w, "t_reduce_ms": round(t, 3), "gflops": round(gf, 1), "flops": "8n^3/3",
            "pct_fp64_peak": round(100 * gf / 1e3 / FP64_PEAK_TFLOPS, 2), "runs": reps}


def cpu_baseline(budget_s=20.0):
    """Time the CPU oracle on a bounded sample of the same workload: one
    factorization of a smaller uniform[-1,1) matrix, sized by cubic
    extrapolation from shorter runs to take about budget_s."""
    import oracle
    import synth
    cores = len(os.sched_getaffinity(0))
    n, t = 1024, 0.0
    for _ in range(4):
        A = synth.uniform(n, seed=1)
        t0 = time.perf_counter()
        oracle.getrf(A, nthreads=cores)
        t = time.perf_counter() - t0
        if t >= 0.4 * budget_s or n >= 16384:
            break
        n = min(16384, max(n + 256, int(n * (budget_s / max(t, 1e-3)) ** (1 / 3)))) // 256 * 256
    out = {"value": round((2.0 / 3.0) * n ** 3 / t / 1e9, 3), "unit": "GFLOP/s", "cores": cores,
           "kind": "oracle",
           "sample": "one FP64 partial-pivoting LU of a uniform[-1,1) %dx%d matrix (%.1f s)" % (n, n, t)}
    out.update(cpu_info())
    return out


def oracle_rate(kind, budget_s=8.0):
    """GFLOP/s of the CPU oracle of one of the other workloads on a bounded
    sample (one run sized by cubic extrapolation to take about budget_s):
    'chol' potrf of the SPD matrix (n^3/3), 'qr' geqrf of a uniform matrix
    (4n^3/3), 'band' the band reduction (8n^3/3, w = 384; single-threaded)."""
    import oracle
    import synth
    cores = len(os.sched_getaffinity(0))
    flops = {"chol": 1.0 / 3.0, "qr": 4.0 / 3.0, "band": 8.0 / 3.0}[kind]
    n, t = 512, 0.0
    for _ in range(5):
        if kind == "chol":
            A = synth.spd(n, seed=7)
            t0 = time.perf_counter()
            oracle.potrf(A, nthreads=cores)
        elif kind == "qr":
            A = synth.uniform(n, seed=11)
            t0 = time.perf_counter()
            oracle.geqrf(A, nthreads=cores)
        else:
            A = synth.uniform(n, seed=13)
            t0 = time.perf_counter()
            oracle.gebrd_band(A, min(384, n))
        t = time.perf_counter() - t0
        if t >= 0.4 * budget_s or n >= 16384:
            break
        n = min(16384, max(n + 256, int(n * (budget_s / max(t, 1e-3)) ** (1 / 3)))) // 256 * 256
    used = 1 if kind == "band" else cores
    what = {"chol": "Cholesky of the SPD", "qr": "Householder QR of a uniform[-1,1)",
            "band": "band reduction (w = %d) of a uniform[-1,1)" % min(384, n)}[kind]
    return {"value": round(flops * n ** 3 / t / 1e9, 3), "unit": "GFLOP/s", "cores": used, "kind": "oracle",
            "sample": "one FP64 %s %dx%d matrix (%.1f s)" % (what, n, n, t)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--b", type=int, default=0)
    ap.add_argument("--depth", type=int, default=-1)
    ap.add_argument("--panel-cus", type=int, default=0)
    ap.add_argument("--taper", type=int, default=0, help="panel taper: 1 on, -1 off, 0 library default")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ir", action="store_true")
    ap.add_argument("--no-chol", action="store_true", help="skip the Cholesky measurement")
    ap.add_argument("--no-qr", action="store_true", help="skip the QR measurement")
    ap.add_argument("--no-band", action="store_true", help="skip the band-reduction measurement")
    ap.add_argument("--band-w", type=int, default=384, help="bandwidth of the band-reduction leg")
    ap.add_argument("--gemm-ceiling", action="store_true",
                    help="also time the library's FP64 trailing GEMM alone on the first update's shape")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the hot path is built and measured on a single MI355X); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1804_07017_amd as lu
    import synth
    lu.load()
    torch.cuda.set_device(0)
    n = args.n
    dev = "cuda"
    g = torch.Generator(device=dev)
    g.manual_seed(1)
    print("bench: generating n=%d inputs" % n, file=sys.stderr, flush=True)
    # the uniform[-1,1) system from the host generators (seed 1): the one the
    # oracle's stored solution and pivot hash belong to
    xo_u, meta_u = oracle_solution(n, "uniform")
    Ah = synth.uniform(n, seed=1)
    if xo_u is not None and not same_matrix(Ah, meta_u["fingerprint"]):
        raise RuntimeError("the regenerated uniform matrix differs from the oracle's")
    A0 = lu.to_device(Ah)
    del Ah
    A = lu.colmajor(n)
    bvec = torch.from_numpy(synth.rhs(n, seed=1)[:, 0].copy()).to(dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    ipiv = torch.zeros(n, dtype=torch.int32, device=dev)
    D = None
    xo = None
    if not args.no_ir:
        # the row-dominant system from the host generators (seed 1): the one
        # the oracle's stored solution belongs to
        xo, meta = oracle_solution(n, "dominant")
        Dh = synth.dominant(n, seed=1)
        if xo is not None and not same_matrix(Dh, meta["fingerprint"]):
            raise RuntimeError("the regenerated row-dominant matrix differs from the oracle's")
        D = lu.to_device(Dh)
        del Dh
        bd = torch.from_numpy(synth.rhs(n, seed=1)[:, 0].copy()).to(dev)
        X = torch.empty(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    sched = None
    if args.b > 0 or args.depth >= 0 or args.panel_cus > 0 or args.taper != 0:
        rc, dflt = lu.lu_schedule_default(n, lu.LU_FP64)
        sched = (args.b, args.depth if args.depth >= 0 else dflt[1], args.panel_cus, args.taper)
    rc, used = lu.lu_schedule_default(n, lu.LU_FP64)
    if sched is not None:
        used = (sched[0] or used[0], sched[1], sched[2] or used[2], sched[3] or used[3])
    taper_on = 1 if used[3] > 0 else 0
    torch.cuda.synchronize()

    def factor_once():
        """FP64 factorization of the pristine matrix; returns its event time (ms)."""
        with torch.cuda.stream(stream):
            A.copy_(A0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            r = lu.lu_factor_ex(A, ipiv, prec=lu.LU_FP64, sched=sched, stream=stream)
            assert r == 0, r
            e1.record(stream)
        stream.synchronize()
        return e0.elapsed_time(e1)

    def step(rec):
        with torch.cuda.stream(stream):
            A.copy_(A0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e2 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            r = lu.lu_factor_ex(A, ipiv, prec=lu.LU_FP64, sched=sched, stream=stream)
            assert r == 0, r
            e1.record(stream)
            x.copy_(bvec)
            r = lu.lu_solve_ex(A, ipiv, x, stream=stream)
            assert r == 0, r
            e2.record(stream)
            ir = None
            if D is not None:
                stream.synchronize()
                t0 = time.perf_counter()
                st, it, res = lu.lu_solve_ir(D, bd, X, prec=lu.LU_MIXED_FP16, max_iter=10, stream=stream)
                stream.synchronize()
                ir = (st, it, res, (time.perf_counter() - t0) * 1e3)
        stream.synchronize()
        rec.append((e0.elapsed_time(e1), e1.elapsed_time(e2), ir))

    warm = []
    for i in range(args.warmup):
        print("bench: warmup step %d" % i, file=sys.stderr, flush=True)
        step(warm)
    rc, info = lu.lu_factor_info()
    if rc != 0:
        print("bench: factorization error %d" % rc, file=sys.stderr)
        sys.exit(1)

    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(recs)
        print("bench: step %d factor %.1f ms solve %.2f ms ir %s" % (i, recs[-1][0], recs[-1][1], recs[-1][2]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # correctness of the last step: HPL residual of the FP64 solve (device GEMV in FP64)
    with torch.no_grad():
        A0r = A0.abs().sum(dim=1).max().item()
        r = (A0 @ x - bvec).abs().max().item()
        hpl = r / (2.0 ** -53 * (A0r * x.abs().max().item() + bvec.abs().max().item()) * n)
    err_vs_oracle = None
    if xo is not None:
        xs = X.cpu().numpy()
        err_vs_oracle = float(np.abs(xs - xo).max() / np.abs(xo).max())
    err64_vs_oracle = pivots_match = None
    if xo_u is not None:
        import hashlib
        err64_vs_oracle = float(np.abs(x.cpu().numpy() - xo_u).max() / np.abs(xo_u).max())
        pivots_match = hashlib.sha256(ipiv.cpu().numpy().astype(np.int32).tobytes()).hexdigest() == \
            meta_u["ipiv_sha256"]

    # untimed passes for the rooflines: the per-launch GEMM timing hook records
    # events around every trailing-GEMM launch of one FP64 factorization and of
    # one mixed-precision factorization (FP32 working copy of the dominant matrix)
    print("bench: roofline passes", file=sys.stderr, flush=True)
    t_mixed = None
    D32 = ip32 = None

    def mixed_factor_once():
        W = D32.clone()
        with torch.cuda.stream(stream):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            r = lu.lu_factor_ex(W, ip32, prec=lu.LU_MIXED_FP16, stream=stream)
            assert r == 0, r
            e1.record(stream)
        stream.synchronize()
        del W
        return e0.elapsed_time(e1)

    if D is not None:
        D32 = D.to(torch.float32)
        ip32 = torch.zeros(n, dtype=torch.int32, device=dev)
        mixed_factor_once()                       # warm-up, not recorded
    lu.lu_k_timing(1)
    t_hooked = factor_once()
    if D is not None:
        t_mixed = mixed_factor_once()
        del D32, ip32
    lu.lu_k_timing(0)
    rc_t, gemm_ms, gemm_flops, gemm_launches = lu.lu_k_timing_read()
    rc_h, half_ms, half_flops, half_bytes, half_launches = lu.lu_k_timing_read_ex(1)

    t_fact = statistics.median(r[0] for r in recs)
    t_solve = statistics.median(r[1] for r in recs)
    flops = (2.0 / 3.0) * n ** 3
    gflops = flops / (t_fact * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(gflops, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FP64 look-ahead LU + 1-RHS solve of the seeded uniform[-1,1) n=%d matrix; mixed "
                               "FP16 LU + FP64 refinement on the seeded row-dominant n=%d matrix" % (n, n),
                   "n": n, "b": used[0], "depth": used[1], "panel_cus": used[2], "taper": taper_on},
        "fp64": {"t_factor_ms": round(t_fact, 3), "t_solve_ms": round(t_solve, 3),
                 "tts_ms": round(t_fact + t_solve, 3), "pct_fp64_peak": round(100 * gflops / 1e3 / FP64_PEAK_TFLOPS, 2),
                 "hpl_resid": hpl, "err_vs_oracle": err64_vs_oracle, "pivots_match_oracle": pivots_match},
    }
    if D is not None:
        irs = [r[2] for r in recs]
        t_ir = statistics.median(i[3] for i in irs)
        mgf = flops / (t_mixed * 1e-3) / 1e9
        out["mixed_ir"] = {"status": irs[-1][0], "iters": irs[-1][1], "hpl_resid": irs[-1][2],
                           "tts_ms": round(t_ir, 3),
                           "speedup_vs_fp64_tts": round((t_fact + t_solve) / t_ir, 3),
                           "effective_gflops": round(flops / (t_ir * 1e-3) / 1e9, 1),
                           "err_vs_oracle": err_vs_oracle,
                           "t_factor_mixed_ms": round(t_mixed, 3),
                           "factor_gflops": round(mgf, 1),
                           "pct_fp16_peak": round(100 * mgf / 1e3 / FP16_PEAK_TFLOPS, 3)}
        if rc_h == 0 and half_launches > 0:
            gbs = half_bytes / (half_ms * 1e-3) / 1e9
            out["mixed_ir"]["roofline"] = {
                "bound": "hbm", "kernel": "gemm_half_sub<_Float16> (mixed trailing update)",
                "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "launches": half_launches, "avg_launch_us": round(half_ms * 1e3 / half_launches, 2),
                "avg_launch_bytes": round(half_bytes / half_launches),
                "mfma_tflops": round(half_flops / (half_ms * 1e-3) / 1e12, 1)}
    if rc_t == 0 and gemm_launches > 0:
        ach = gemm_flops / (gemm_ms * 1e-3) / 1e12
        traffic = None
        if (GEMM_TRAFFIC["n"], GEMM_TRAFFIC["b"], GEMM_TRAFFIC["depth"], GEMM_TRAFFIC["taper"]) == \
                (n, used[0], used[1], taper_on) and \
                GEMM_TRAFFIC["gemm_source_sha256_16"] == gemm_source_hash():
            traffic = GEMM_TRAFFIC["bytes_per_launch"]
        out["roofline"] = {"bound": "mfma", "kernel": "gemm_nn_sub<double,16> (trailing update)",
                           "achieved": round(ach, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": round(ach / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                           "traffic_unit": "bytes per launch",
                           "algorithmic_bytes_per_launch": round(gemm_algorithmic_bytes(lu, n, used[0], used[1],
                                                                                        taper_on)),
                           "launches": gemm_launches,
                           "avg_launch_us": round(gemm_ms * 1e3 / gemm_launches, 2),
                           "avg_launch_gflop": round(gemm_flops / gemm_launches / 1e9, 3),
                           "hooked_factor_ms": round(t_hooked, 3)}
    if args.gemm_ceiling:
        # the library's trailing GEMM alone on the first update's shape
        bb = used[0]
        M = N = n - bb
        Am = lu.colmajor(M, bb)
        Am.uniform_(-1.0, 1.0, generator=g)
        Bm = lu.colmajor(bb, N)
        Bm.uniform_(-1.0, 1.0, generator=g)
        ts = []
        for rep in range(6):
            with torch.cuda.stream(stream):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                r = lu.lu_k_gemm(Am, Bm, A[:M, :N], prec=lu.LU_FP64, stream=stream)
                assert r == 0, r
                e1.record(stream)
            stream.synchronize()
            if rep:
                ts.append(e0.elapsed_time(e1))
        tc = statistics.median(ts)
        tf = 2.0 * M * N * bb / (tc * 1e-3) / 1e12
        out["gemm_ceiling"] = {"kernel": "gemm_nn_sub<double,16> alone", "m": M, "n": N, "k": bb,
                               "ms": round(tc, 3), "tflops": round(tf, 2),
                               "frac_of_peak": round(tf / FP64_PEAK_TFLOPS, 4),
                               "lu_pct_of_ceiling": round(100 * gflops / 1e3 / tf, 2)}
        del Am, Bm
    if not args.no_chol:
        out["cholesky"] = cholesky_leg(lu, n, args.steps, A0, A)
    if not args.no_qr:
        out["qr"] = qr_leg(lu, n, args.steps, A0, A)
    if not args.no_band:
        out["band"] = band_leg(lu, n, args.band_w, args.steps, A0, A)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
        for key, kind in (("cholesky", "chol"), ("qr", "qr"), ("band", "band")):
            if key in out:
                print("bench: cpu oracle (%s)" % kind, file=sys.stderr, flush=True)
                out[key]["cpu_oracle"] = oracle_rate(kind)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
