"""Host-side checks of the native library (no GPU): it loads, exports every
symbol the headers declare, rejects illegal arguments before touching the
device, and the schedule planner builds sound look-ahead task graphs."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_1804_07017_amd as lu
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:int|void)\s+((?:lu|chol|qr|band)_\w+)\s*\(", txt, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = lu.load()
    declared = _declared_symbols()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(lu.exported_symbols())


def test_argument_errors_before_any_device_call():
    lib = lu.load()
    assert lib.lu_factor(-1, None, 1, None, None) == -1
    assert lib.lu_factor(4, None, 4, None, None) == -2
    assert lib.lu_factor(4, 8, 3, 8, None) == -3
    assert lib.lu_factor(4, 8, 4, None, None) == -4
    assert lib.lu_factor(0, None, 1, None, None) == 0
    assert lib.lu_factor_ex(4, 8, 4, 7, 8, None, None, None) == -5
    bad = lu.Schedule(100, 1, 16)
    import ctypes
    assert lib.lu_factor_ex(4, 8, 4, 0, 8, ctypes.byref(bad), None, None) == -6
    bad = lu.Schedule(64, 3, 16)
    assert lib.lu_factor_ex(4, 8, 4, 0, 8, ctypes.byref(bad), None, None) == -6
    assert lib.lu_solve(-1, 1, None, None, None) == -1
    assert lib.lu_solve(4, -1, None, None, None) == -2
    assert lib.lu_solve_ex(4, 1, 8, 2, 8, 8, 4, None) == -4
    assert lib.lu_solve_ex(4, 1, 8, 4, 8, 8, 2, None) == -7
    it = ctypes.c_int(0)
    res = ctypes.c_double(0)
    assert lib.lu_solve_ir(4, 1, 8, 4, 8, 4, 8, 4, 9, 5, ctypes.byref(it), ctypes.byref(res), None) == -9
    assert lib.lu_solve_ir(4, 1, 8, 4, 8, 4, 8, 4, 2, 0, ctypes.byref(it), ctypes.byref(res), None) == -10
    assert lib.lu_solve_ir(0, 1, None, 1, None, 1, None, 1, 2, 5, ctypes.byref(it), ctypes.byref(res), None) == 0
    assert lib.lu_k_panel(0, 4, 8, 8, 4, 8, 0, None, None) == -3
    assert lib.lu_k_gemm(0, 4, 4, 4, 8, 2, 8, 4, 8, 4, None) == -6
    # Cholesky, QR and the band reduction check their arguments the same way
    assert lib.chol_factor(-1, None, 1, None) == -1
    assert lib.chol_factor(4, None, 4, None) == -2
    assert lib.chol_factor(4, 8, 3, None) == -3
    assert lib.chol_factor(0, None, 1, None) == 0
    assert lib.chol_factor_ex(4, 8, 4, ctypes.byref(lu.Schedule(100, 1, 16)), None, None) == -4
    assert lib.qr_factor(-1, 1, 8, 1, 8, None) == -1
    assert lib.qr_factor(3, 4, 8, 4, 8, None) == -2
    assert lib.qr_factor(4, 4, None, 4, 8, None) == -3
    assert lib.qr_factor(4, 4, 8, 3, 8, None) == -4
    assert lib.qr_factor(4, 4, 8, 4, None, None) == -5
    assert lib.qr_factor(0, 0, None, 1, None, None) == 0
    assert lib.qr_factor_ex(4, 4, 8, 4, 8, ctypes.byref(lu.Schedule(100, 1, 16)), None) == -6
    assert lib.qr_factor_ex(4, 4, 8, 4, 8, ctypes.byref(lu.Schedule(128, 3, 16)), None) == -6
    assert lib.band_reduce(-1, 8, 1, 2, 8, 8, None) == -1
    assert lib.band_reduce(4, None, 4, 2, 8, 8, None) == -2
    assert lib.band_reduce(4, 8, 3, 2, 8, 8, None) == -3
    assert lib.band_reduce(4, 8, 4, 0, 8, 8, None) == -4
    assert lib.band_reduce(4, 8, 4, 385, 8, 8, None) == -4
    assert lib.band_reduce(4, 8, 4, 2, None, 8, None) == -5
    assert lib.band_reduce(4, 8, 4, 2, 8, None, None) == -6
    assert lib.band_reduce(0, None, 1, 2, None, None, None) == 0


def test_selector_file_errors(tmp_path):
    assert lu.lu_selector_load(tmp_path / "missing.bin") < 0
    p = tmp_path / "bad.bin"
    p.write_bytes(b"not a weights file")
    assert lu.lu_selector_load(p) < 0


# ------------------------------------------------------------- plan checks
def _uniform_starts(n, b):
    return list(range(0, n, b)) + [n]


def _access(t, starts):
    """(write columns, read columns, ipiv written, ipiv read) of a task."""
    w = set(range(t["col_begin"], t["col_end"]))
    r = set()
    ipw = ipr = None
    if t["kind"] == lu.LU_TASK_PANEL:
        ipw = t["step"]
    elif t["kind"] == lu.LU_TASK_UPDATE:
        k = t["step"]
        r = set(range(starts[k], starts[k + 1]))
        ipr = {k}
    elif t["kind"] == lu.LU_TASK_LPERM:
        ipr = set(range(len(starts) - 1))          # every panel's pivots
    else:
        ipr = {t["step"]}
    return w, r, ipw, ipr or set()


def _happens_before(tasks):
    T = len(tasks)
    before = [set() for _ in range(T)]
    last = {s: None for s in range(3)}
    for i, t in enumerate(tasks):
        s = t["stream"]
        if last[s] is not None:
            before[i] |= before[last[s]] | {last[s]}
        for wv in t["waits"]:
            before[i] |= before[wv] | {wv}
        last[s] = i
    return before


def _check_plan(n, starts, depth, tasks, swaps=1):
    N = len(starts) - 1
    # every panel factored once; every (step, column) pair of the trailing
    # matrix updated exactly once; every left swap applied once
    panels = [t["step"] for t in tasks if t["kind"] == lu.LU_TASK_PANEL]
    assert sorted(panels) == list(range(N))
    for t in tasks:
        if t["kind"] == lu.LU_TASK_PANEL:
            assert (t["col_begin"], t["col_end"]) == (starts[t["step"]], starts[t["step"] + 1])
    cover = {}
    for t in tasks:
        if t["kind"] == lu.LU_TASK_UPDATE:
            for c in range(t["col_begin"], t["col_end"]):
                cover[(t["step"], c)] = cover.get((t["step"], c), 0) + 1
    for k in range(N):
        for c in range(starts[k + 1], n):
            assert cover.get((k, c)) == 1, (k, c)
    assert len(cover) == sum(n - starts[k + 1] for k in range(N))
    lswaps = sorted((t["step"], t["col_begin"], t["col_end"]) for t in tasks if t["kind"] == lu.LU_TASK_LSWAP)
    lperms = [(t["step"], t["col_begin"], t["col_end"], t["stream"]) for t in tasks if t["kind"] == lu.LU_TASK_LPERM]
    if swaps == 1:
        assert lswaps == [(k, 0, starts[k]) for k in range(1, N)] and not lperms
    else:
        # one deferred permutation of every finished panel, the last task
        assert not lswaps
        assert lperms == ([(N - 1, 0, starts[N - 1], 0)] if N >= 2 else [])
        if N >= 2:
            assert tasks[-1]["kind"] == lu.LU_TASK_LPERM
    if depth == 0:
        assert all(t["stream"] == 0 for t in tasks)
    else:
        assert all(t["stream"] == 1 for t in tasks if t["kind"] == lu.LU_TASK_PANEL)
        assert all(t["stream"] == 2 for t in tasks if t["kind"] == lu.LU_TASK_LSWAP)
    for t in tasks:
        # at most one wait per other stream, each on an earlier task of another stream
        assert len(t["waits"]) == len({tasks[w]["stream"] for w in t["waits"]})
        assert all(tasks[w]["stream"] != t["stream"] for w in t["waits"])
    # race freedom: tasks not ordered by happens-before touch disjoint data
    hb = _happens_before(tasks)
    acc = [_access(t, starts) for t in tasks]
    for i in range(len(tasks)):
        for j in range(i):
            if j in hb[i]:
                continue
            wi, ri, pwi, pri = acc[i]
            wj, rj, pwj, prj = acc[j]
            assert not (wi & wj) and not (wi & rj) and not (ri & wj), (tasks[j], tasks[i])
            assert pwi is None or (pwi not in prj and pwi != pwj)
            assert pwj is None or pwj not in pri


@pytest.mark.parametrize("n,b,depth", [(10, 4, 0), (10, 4, 1), (13, 4, 2), (64, 16, 1), (70, 16, 2),
                                       (33, 8, 2), (8, 8, 1), (5, 8, 2), (100, 32, 1)])
def test_plan_is_race_free_and_complete(n, b, depth):
    rc, tasks = lu.lu_plan_build(n, b, depth)
    assert rc == len(tasks) > 0
    _check_plan(n, _uniform_starts(n, b), depth, tasks)
    # the same plan from explicit uniform boundaries
    rc2, tasks2 = lu.lu_plan_build_panels(n, _uniform_starts(n, b), depth)
    assert rc2 == rc and tasks2 == tasks


@pytest.mark.parametrize("starts,depth", [([0, 8, 12, 14, 15], 1), ([0, 8, 12, 14, 15], 2),
                                          ([0, 3, 11, 12, 20, 21], 2), ([0, 16, 24, 28, 30, 31], 0),
                                          ([0, 1], 2), ([0, 1, 2], 2)])
def test_plan_with_variable_panels_is_race_free_and_complete(starts, depth):
    n = starts[-1]
    rc, tasks = lu.lu_plan_build_panels(n, starts, depth)
    assert rc == len(tasks) > 0
    _check_plan(n, starts, depth, tasks)


def test_taper_boundaries():
    """The early-termination taper: panels never wider than b, 128 wide once
    the trailing size drops to the precision's threshold, exact cover."""
    thresholds = {0: 12288, 1: 16384, 2: 16384, 3: 16384}
    for prec, t128 in thresholds.items():
        for n, b in [(32768, 256), (12000, 256), (20000, 512), (45000, 512), (3000, 64), (700, 128)]:
            rc, st = lu.lu_plan_panels(n, b, 1, prec)
            assert rc == len(st) - 1 and st[0] == 0 and st[-1] == n
            for j in range(rc):
                w, r = st[j + 1] - st[j], n - st[j]
                want = b if r > t128 else min(b, 128)
                assert w == min(want, r), (prec, n, b, j, w)
            # taper off: uniform b
            rc0, st0 = lu.lu_plan_panels(n, b, -1, prec)
            assert st0 == _uniform_starts(n, b)
    assert lu.lu_plan_panels(0, 256, 1, 0) == (0, [])
    assert lu.lu_plan_panels(-1, 256, 1, 0)[0] == -1
    assert lu.lu_plan_panels(10, 0, 1, 0)[0] == -2
    assert lu.lu_plan_panels(10, 4, 1, 7)[0] == -4
    assert lu.lu_plan_panels(100, 8, 1, 0, max_starts=5)[0] == -5
    # boundaries that are not strictly increasing from 0 to n are rejected
    assert lu.lu_plan_build_panels(10, [0, 5, 5, 10], 1)[0] == -4
    assert lu.lu_plan_build_panels(10, [0, 5, 9], 1)[0] == -4
    assert lu.lu_plan_build_panels(10, [1, 5, 10], 1)[0] == -4
    assert lu.lu_plan_build_panels(10, [0, 5, 10], 3)[0] == -3


def _run_task(A, ipiv, t, starts, n):
    """Execute one plan task on the numpy matrix A (FP64) in place."""
    k = t["step"]
    c0, c1 = t["col_begin"], t["col_end"]
    if t["kind"] == lu.LU_TASK_PANEL:
        j0, j1 = c0, c1
        for d in range(j0, j1):
            p = d + int(np.argmax(np.abs(A[d:, d])))
            ipiv[d] = p
            if p != d:
                A[[d, p], j0:j1] = A[[p, d], j0:j1]
            if A[d, d] != 0:
                A[d + 1:, d] /= A[d, d]
            A[d + 1:, d + 1:j1] -= np.outer(A[d + 1:, d], A[d, d + 1:j1])
    elif t["kind"] == lu.LU_TASK_UPDATE:
        kb, w = starts[k], starts[k + 1] - starts[k]
        for d in range(kb, kb + w):
            p = ipiv[d]
            if p != d:
                A[[d, p], c0:c1] = A[[p, d], c0:c1]
        L11 = np.tril(A[kb:kb + w, kb:kb + w], -1) + np.eye(w)
        A[kb:kb + w, c0:c1] = np.linalg.solve(L11, A[kb:kb + w, c0:c1])
        A[kb + w:, c0:c1] -= A[kb + w:, kb:kb + w] @ A[kb:kb + w, c0:c1]
    elif t["kind"] == lu.LU_TASK_LPERM:
        # every panel j >= 1's interchanges on the columns left of it
        for d in range(starts[1], n):
            p = ipiv[d]
            j = max(i for i in range(len(starts) - 1) if starts[i] <= d)
            if p != d:
                A[[d, p], 0:starts[j]] = A[[p, d], 0:starts[j]]
    else:
        kb, w = starts[k], starts[k + 1] - starts[k]
        for d in range(kb, kb + w):
            p = ipiv[d]
            if p != d:
                A[[d, p], c0:c1] = A[[p, d], c0:c1]


def _random_legal_order(tasks, rng):
    q = {s: [i for i, t in enumerate(tasks) if t["stream"] == s] for s in range(3)}
    done = set()
    order = []
    while any(q.values()):
        ready = [s for s in range(3) if q[s] and all(w in done for w in tasks[q[s][0]]["waits"])]
        assert ready, "plan deadlocks"
        s = ready[rng.integers(len(ready))]
        i = q[s].pop(0)
        done.add(i)
        order.append(i)
    return order


@pytest.mark.parametrize("n,starts,depth", [(24, 4, 1), (30, 8, 2), (37, 8, 1), (37, 8, 2), (40, 8, 0),
                                            (37, [0, 12, 20, 26, 30, 33, 35, 36, 37], 2),
                                            (37, [0, 12, 20, 26, 30, 33, 35, 36, 37], 1)])
def test_plan_executes_to_the_oracle_result_in_any_legal_order(n, starts, depth):
    import oracle
    import synth
    A0 = np.array(synth.uniform(n, seed=n), order="F")
    if isinstance(starts, int):
        rc, tasks = lu.lu_plan_build(n, starts, depth)
        starts = _uniform_starts(n, starts)
    else:
        rc, tasks = lu.lu_plan_build_panels(n, starts, depth)
    results = []
    rng = np.random.default_rng(0)
    for trial in range(4):
        A = A0.copy()
        ipiv = np.zeros(n, dtype=np.int64)
        order = range(len(tasks)) if trial == 0 else _random_legal_order(tasks, rng)
        for i in order:
            _run_task(A, ipiv, tasks[i], starts, n)
        results.append((A, ipiv))
    for A, ipiv in results[1:]:
        assert np.array_equal(A, results[0][0]) and np.array_equal(ipiv, results[0][1])
    LU, ip, info = oracle.getrf(A0)
    assert np.array_equal(results[0][1], ip)
    assert np.abs(results[0][0] - LU).max() <= 1e-10 * max(1.0, np.abs(LU).max())


def _run_qr_task(A, tau, t, starts):
    """One task of the interchange-free plan as the QR executor runs it:
    PANEL(k) Householder QR of rows kb.. of the panel's columns; UPDATE(k, c0,
    c1) the panel's block reflector applied to those rows of columns c0..c1."""
    k = t["step"]
    kb, w = starts[k], starts[k + 1] - starts[k]
    if t["kind"] == lu.LU_TASK_PANEL:
        P = A[kb:, kb:kb + w]
        for j in range(w):
            alpha = P[j, j]
            s = float(np.dot(P[j + 1:, j], P[j + 1:, j]))
            if s == 0.0:
                continue
            beta = -np.sqrt(alpha * alpha + s) if alpha >= 0.0 else np.sqrt(alpha * alpha + s)
            tau[kb + j] = (beta - alpha) / beta
            P[j + 1:, j] *= 1.0 / (alpha - beta)
            P[j, j] = beta
            v = np.concatenate(([1.0], P[j + 1:, j]))
            P[j:, j + 1:] -= tau[kb + j] * np.outer(v, v @ P[j:, j + 1:])
    else:
        assert t["kind"] == lu.LU_TASK_UPDATE
        c0, c1 = t["col_begin"], t["col_end"]
        V = np.tril(A[kb:, kb:kb + w], -1)
        V[np.arange(w), np.arange(w)] = 1.0
        for j in range(w):                       # H_0 ... H_{w-1} applied in order: Q^T C
            v = V[:, j]
            C = A[kb:, c0:c1]
            C -= tau[kb + j] * np.outer(v, v @ C)


@pytest.mark.parametrize("starts,depth", [([0, 8, 16, 24, 30], 1), ([0, 8, 16, 24, 30], 2),
                                          ([0, 4, 12, 13, 20], 2), ([0, 10, 20], 0)])
def test_interchange_free_plan_executes_to_the_qr_oracle(starts, depth):
    """The task list the QR and Cholesky executors use: no LSWAP tasks, and
    executed in random legal orders (stream order kept) it gives the QR
    oracle's factorization."""
    n = starts[-1]
    rc, tasks = lu.lu_plan_build_panels_ex(n, starts, depth, 0)
    assert rc == len(tasks) > 0
    assert not any(t["kind"] == lu.LU_TASK_LSWAP for t in tasks)
    rc1, tasks1 = lu.lu_plan_build_panels_ex(n, starts, depth, 1)
    assert (rc1, tasks1) == lu.lu_plan_build_panels(n, starts, depth)
    A0 = synth.uniform(n, seed=n + depth)
    oF, otau = oracle.geqrf(A0)
    rng = np.random.default_rng(depth + 7)
    for _ in range(3):
        A = np.array(A0, order="F", copy=True)
        tau = np.zeros(n)
        for i in _random_legal_order(tasks, rng):
            _run_qr_task(A, tau, tasks[i], starts)
        assert np.abs(A - oF).max() <= 1e-12
        assert np.abs(tau - otau).max() <= 1e-13


def test_refinement_outcome_mapping():
    """lu_solve_ir's final status (host logic, no device call): a singular FP64
    factor is an error, a non-finite residual is reported as such, a residual
    above the HPL bound of 16 is flagged, and the fall-back is distinguished
    from plain convergence."""
    lib = lu.load()
    nan = float("nan")
    assert lib.lu_ir_outcome(0, 0, 0.05) == lu.LU_IR_OK
    assert lib.lu_ir_outcome(0, 0, 16.0) == lu.LU_IR_OK
    assert lib.lu_ir_outcome(0, 1, 0.05) == lu.LU_IR_FELL_BACK
    assert lib.lu_ir_outcome(0, 0, 16.5) == lu.LU_IR_RESID_HIGH
    assert lib.lu_ir_outcome(0, 1, 1e30) == lu.LU_IR_RESID_HIGH
    assert lib.lu_ir_outcome(0, 0, nan) == lu.LU_ERR_NONFINITE
    assert lib.lu_ir_outcome(0, 1, float("inf")) == lu.LU_IR_RESID_HIGH
    assert lib.lu_ir_outcome(7, 0, 0.0) == lu.LU_ERR_SINGULAR
    assert lib.lu_ir_outcome(1, 1, nan) == lu.LU_ERR_SINGULAR


def test_garbage_interchange_lists_stay_in_bounds():
    """The trailing kernels read a panel's composed interchange list through
    the functions lu_k_moves_check runs on the host: whatever the list holds
    (an empty one from a panel that gave up at a barrier time-out, stale or
    random words), every kept move addresses rows inside the block, so the
    kernels' LDS indices and matrix rows stay in range."""
    lib = lu.load()
    MAXW = 512
    LEN = 2 + 4 * MAXW
    rng = np.random.default_rng(7)
    out = np.zeros(4 * MAXW, dtype=np.int32)
    # an empty list keeps nothing
    mv = np.zeros(LEN, dtype=np.int32)
    assert lib.lu_k_moves_check(mv.ctypes.data, 256, 1000, out.ctypes.data) == 0
    for trial in range(300):
        w = int(rng.integers(1, MAXW + 1))
        m = int(rng.integers(w, 70000))
        kind = trial % 3
        if kind == 0:          # random words, including huge and negative counts
            mv = rng.integers(-2 ** 31, 2 ** 31 - 1, LEN, dtype=np.int64).astype(np.int32)
        elif kind == 1:        # plausible counts, rows slightly out of range
            mv = rng.integers(-3, m + 3, LEN).astype(np.int32)
            mv[0] = rng.integers(0, 2 * MAXW)
            mv[1] = rng.integers(0, 2 * MAXW)
        else:                  # counts beyond the width
            mv = rng.integers(0, m, LEN).astype(np.int32)
            mv[0] = MAXW + 5
            mv[1] = -1
        r = lib.lu_k_moves_check(mv.ctypes.data, w, m, out.ctypes.data)
        assert r >= 0
        nt, ne = r >> 16, r & 0xFFFF
        assert nt <= w and ne <= w
        top = out[:2 * nt].reshape(-1, 2)
        ext = out[2 * nt:2 * (nt + ne)].reshape(-1, 2)
        assert np.all((top[:, 0] >= 0) & (top[:, 0] < w) & (top[:, 1] >= 0) & (top[:, 1] < m))
        assert np.all((ext[:, 0] >= w) & (ext[:, 0] < m) & (ext[:, 1] >= 0) & (ext[:, 1] < w))
    # a well-formed list from the composition is kept whole
    w, m = 4, 10
    piv = np.array([7, 1, 9, 3], dtype=np.int32)      # swaps (0,7), (2,9)
    mv = np.zeros(LEN, dtype=np.int32)
    mv[0], mv[1] = 2, 2
    mv[2:6] = [0, 7, 2, 9]
    mv[2 + 2 * MAXW:2 + 2 * MAXW + 4] = [7, 0, 9, 2]
    r = lib.lu_k_moves_check(mv.ctypes.data, w, m, out.ctypes.data)
    assert (r >> 16, r & 0xFFFF) == (2, 2)
    assert out[:8].tolist() == [0, 7, 2, 9, 7, 0, 9, 2]


@pytest.mark.parametrize("n,starts,depth", [(24, 4, 1), (30, 8, 2), (37, 8, 0), (37, 8, 2),
                                            (37, [0, 12, 20, 26, 30, 33, 35, 36, 37], 2),
                                            (37, [0, 12, 20, 26, 30, 33, 35, 36, 37], 1), (5, [0, 5], 1)])
def test_deferred_left_interchanges_plan(n, starts, depth):
    """The plan with the left interchanges deferred to one final LPERM task
    (what the library runs when a column fits its permutation kernel) is
    complete and race-free, and executed in random legal orders it gives the
    oracle's factors and pivots."""
    import oracle
    import synth
    if isinstance(starts, int):
        starts = _uniform_starts(n, starts)
    rc, tasks = lu.lu_plan_build_panels_ex(n, starts, depth, 2)
    assert rc == len(tasks) > 0
    _check_plan(n, starts, depth, tasks, swaps=2)
    A0 = np.array(synth.uniform(n, seed=n + 1), order="F")
    rng = np.random.default_rng(1)
    results = []
    for trial in range(3):
        A = A0.copy()
        ipiv = np.zeros(n, dtype=np.int64)
        order = range(len(tasks)) if trial == 0 else _random_legal_order(tasks, rng)
        for i in order:
            _run_task(A, ipiv, tasks[i], starts, n)
        results.append((A, ipiv))
    for A, ipiv in results[1:]:
        assert np.array_equal(A, results[0][0]) and np.array_equal(ipiv, results[0][1])
    LU, ip, info = oracle.getrf(A0)
    assert np.array_equal(results[0][1], ip)
    assert np.abs(results[0][0] - LU).max() <= 1e-10 * max(1.0, np.abs(LU).max())


def test_deferred_permutation_composition_matches_sequential_swaps():
    """The composition the permutation kernel computes, modelled in numpy from
    its description: for panel k, inv starts as the identity on rows >= r0 =
    s_k+1; the panels j = N-1 down to k+1 each set inv[src] = inv[dst] for
    their composed moves (new[dst] = old[src], here built from ipiv by
    simulating the panel's interchanges); the column is written new[inv[i]] =
    old[i].  It must equal applying ipiv[r0:] row swaps one by one."""
    rng = np.random.default_rng(5)
    for trial in range(30):
        n = int(rng.integers(8, 60))
        cuts = sorted(set(int(x) for x in rng.integers(1, n, int(rng.integers(1, 6)))))
        starts = [0] + cuts + [n]
        ipiv = np.array([int(rng.integers(d, n)) for d in range(n)])
        N = len(starts) - 1

        def moves_of(j):
            # new[dst] = old[src] for the rows the panel's interchanges move
            idx = np.arange(n)
            for d in range(starts[j], starts[j + 1]):
                p = ipiv[d]
                idx[[d, p]] = idx[[p, d]]
            return [(r, idx[r]) for r in range(n) if idx[r] != r]

        for k in range(N - 1):
            r0 = starts[k + 1]
            col = rng.standard_normal(n)
            want = col.copy()
            for d in range(r0, n):
                p = ipiv[d]
                want[[d, p]] = want[[p, d]]
            inv = np.arange(n - r0)
            for j in range(N - 1, k, -1):
                mv = moves_of(j)
                old = inv.copy()
                for dst, src in mv:
                    inv[src - r0] = old[dst - r0]
            got = col.copy()
            seg = col[r0:].copy()
            got[r0 + inv] = seg
            assert np.array_equal(got, want), (trial, k)
