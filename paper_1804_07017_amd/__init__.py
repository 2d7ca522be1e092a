"""Python binding of the MI355X look-ahead LU library (liblu_mi355x.so).

Thin ctypes marshalling over the C ABI in ``include/lu.h``, ``lu_plan.h`` and
``lu_kernels.h``: every computation runs in the library's HIP kernels.  The
functions keep the C names.  Matrices are column-major device tensors (torch
tensors with ``stride(0) == 1``; ``stride(1)`` is the leading dimension);
``colmajor`` and ``to_device`` build such tensors.  PyTorch supplies device
memory and streams only.

If the native library has not been built, ``load()`` raises: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblu_mi355x.so")

LU_FP64, LU_FP32, LU_MIXED_FP16, LU_MIXED_BF16 = 0, 1, 2, 3
LU_ERR_HIP, LU_ERR_BARRIER, LU_ERR_NOMEM, LU_ERR_UNSUPPORTED, LU_ERR_NONFINITE = -100, -101, -102, -103, -104
LU_NOALLOC_MAX_N = 65536
LU_ERR_SINGULAR = -105
LU_IR_OK, LU_IR_FELL_BACK, LU_IR_RESID_HIGH = 0, 1, 2
LU_TASK_PANEL, LU_TASK_UPDATE, LU_TASK_LSWAP, LU_TASK_LPERM = 0, 1, 2, 3
SELECTOR_PARAMS = 490

_lib = None


class Schedule(ctypes.Structure):
    _fields_ = [("b", ctypes.c_int), ("depth", ctypes.c_int), ("panel_cus", ctypes.c_int),
                ("taper", ctypes.c_int)]


class PlanTask(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("step", ctypes.c_int), ("col_begin", ctypes.c_int),
                ("col_end", ctypes.c_int), ("stream", ctypes.c_int), ("nwait", ctypes.c_int),
                ("wait", ctypes.c_int * 2), ("record", ctypes.c_int)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "lu_factor": (_I, [_I, _P, _I, _P, _P]),
    "lu_factor_ex": (_I, [_I, _P, _I, _I, _P, ctypes.POINTER(Schedule), _P, _P]),
    "lu_factor_info": (_I, [ctypes.POINTER(_I)]),
    "lu_schedule_default": (_I, [_I, _I, ctypes.POINTER(Schedule)]),
    "lu_solve": (_I, [_I, _I, _P, _P, _P]),
    "lu_solve_ex": (_I, [_I, _I, _P, _I, _P, _P, _I, _P]),
    "lu_solve_noalloc": (_I, [_I, _I, _P, _I, _P, _P, _I, _P]),
    "lu_solve_ir": (_I, [_I, _I, _P, _I, _P, _I, _P, _I, _I, _I, ctypes.POINTER(_I),
                         ctypes.POINTER(ctypes.c_double), _P]),
    "lu_selector_load": (_I, [ctypes.c_char_p]),
    "lu_selector_predict": (_I, [_I, _I, ctypes.POINTER(Schedule)]),
    "lu_selector_train": (_I, [_P, _P, _I, _I, ctypes.c_float, _I, _P]),
    "lu_selector_save": (_I, [ctypes.c_char_p]),
    "lu_selector_get_params": (_I, [_P, _I]),
    "lu_selector_set_params": (_I, [_P, _I, _I, _I]),
    "lu_selector_grad": (_I, [_P, _P, _I, _P, _P]),
    "lu_release": (None, []),
    "lu_plan_build": (_I, [_I, _I, _I, ctypes.POINTER(PlanTask), _I]),
    "chol_factor": (_I, [_I, _P, _I, _P]),
    "chol_factor_ex": (_I, [_I, _P, _I, ctypes.POINTER(Schedule), _P, _P]),
    "chol_solve": (_I, [_I, _I, _P, _I, _P, _I, _P]),
    "qr_factor": (_I, [_I, _I, _P, _I, _P, _P]),
    "qr_factor_ex": (_I, [_I, _I, _P, _I, _P, ctypes.POINTER(Schedule), _P]),
    "band_reduce": (_I, [_I, _P, _I, _I, _P, _P, _P]),
    "lu_plan_panels": (_I, [_I, _I, _I, _I, ctypes.POINTER(_I), _I]),
    "lu_plan_build_panels": (_I, [_I, ctypes.POINTER(_I), _I, _I, ctypes.POINTER(PlanTask), _I]),
    "lu_plan_build_panels_ex": (_I, [_I, ctypes.POINTER(_I), _I, _I, _I, ctypes.POINTER(PlanTask), _I]),
    "lu_k_panel": (_I, [_I, _I, _I, _P, _I, _P, _I, _P, _P]),
    "lu_k_update": (_I, [_I, _I, _I, _I, _P, _I, _P, _P, _I, _P]),
    "lu_k_gemm": (_I, [_I, _I, _I, _I, _P, _I, _P, _I, _P, _I, _P]),
    "lu_k_laswp": (_I, [_I, _I, _I, _I, _P, _P, _I, _P]),
    "lu_k_probe_mfma_f64": (_I, [_P, _P]),
    "lu_ir_outcome": (_I, [_I, _I, ctypes.c_double]),
    "lu_k_moves_check": (_I, [_P, _I, _I, _P]),
    "lu_k_xcd_probe": (_I, [_P]),
    "lu_k_timing": (_I, [_I]),
    "lu_k_timing_read": (_I, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(_I)]),
    "lu_k_timing_read_ex": (_I, [_I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I)]),
}


def load():
    """Load liblu_mi355x.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblu_mi355x.so not built: run __graft_entry__.build() "
                              "(or python paper_1804_07017_amd/build.py)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS)


# ------------------------------------------------------------------ helpers
def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ld(t):
    """Leading dimension of a column-major 2-D tensor (or 1-D vector)."""
    if t.dim() == 1:
        return max(1, t.shape[0])
    if t.stride(0) != 1 and t.shape[0] > 1:
        raise ValueError("column-major tensor expected (stride(0) == 1)")
    return max(1, t.stride(1), t.shape[0]) if t.shape[1] > 1 else max(1, t.shape[0])


def colmajor(n_rows, n_cols=None, lda=None, dtype=None, device="cuda"):
    """Uninitialised column-major (n_rows x n_cols) tensor with leading dimension lda."""
    import torch
    n_cols = n_rows if n_cols is None else n_cols
    lda = n_rows if lda is None else lda
    dtype = torch.float64 if dtype is None else dtype
    buf = torch.empty((max(n_cols, 1), max(lda, 1)), dtype=dtype, device=device)
    return buf.t()[:n_rows, :n_cols]


def to_device(a, dtype=None, device="cuda", lda=None):
    """numpy (any order) -> column-major device tensor with the same values."""
    import numpy as np
    import torch
    a = np.asarray(a)
    if a.ndim == 1:
        return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype or torch.float64)
    t = colmajor(a.shape[0], a.shape[1], lda=lda, dtype=dtype or torch.from_numpy(a[:0, :0].copy()).dtype,
                 device=device)
    t.copy_(torch.from_numpy(np.asfortranarray(a)))
    return t


def to_host(t):
    """Column-major device tensor -> Fortran-ordered numpy array."""
    import numpy as np
    a = t.detach().cpu().numpy()
    return np.asfortranarray(a)


def _sched(sched):
    if sched is None:
        return None
    if isinstance(sched, Schedule):
        return ctypes.byref(sched)
    b, d, p = sched[:3]
    taper = sched[3] if len(sched) > 3 else 0
    return ctypes.byref(Schedule(int(b), int(d), int(p), int(taper)))


# ------------------------------------------------------------------ C ABI
def lu_factor(A, ipiv, stream=None):
    n = A.shape[0]
    return load().lu_factor(n, _ptr(A), _ld(A), _ptr(ipiv), _stream(stream))


def lu_factor_ex(A, ipiv, prec=LU_FP64, sched=None, d_info=None, stream=None, n=None):
    n = A.shape[0] if n is None else n
    return load().lu_factor_ex(n, _ptr(A), _ld(A), int(prec), _ptr(ipiv), _sched(sched), _ptr(d_info),
                               _stream(stream))


def chol_factor(A, stream=None, n=None):
    """Cholesky A = L L^T (lower triangle, FP64) of the column-major device matrix A."""
    n = A.shape[0] if n is None else n
    return load().chol_factor(n, _ptr(A), _ld(A), _stream(stream))


def chol_factor_ex(A, sched=None, d_info=None, stream=None, n=None):
    n = A.shape[0] if n is None else n
    return load().chol_factor_ex(n, _ptr(A), _ld(A), _sched(sched), _ptr(d_info), _stream(stream))


def chol_solve(L, B, stream=None, n=None):
    """B <- (L L^T)^-1 B with the factor of chol_factor (device tensors, column-major)."""
    n = L.shape[0] if n is None else n
    nrhs = 1 if B.dim() == 1 else B.shape[1]
    return load().chol_solve(n, nrhs, _ptr(L), _ld(L), _ptr(B), _ld(B) if B.dim() > 1 else max(1, n),
                             _stream(stream))


def qr_factor(A, tau, sched=None, stream=None):
    """Householder QR of the column-major device matrix A (m x n, m >= n) in place; tau (n,) device."""
    m, n = A.shape
    if sched is None:
        return load().qr_factor(m, n, _ptr(A), _ld(A), _ptr(tau), _stream(stream))
    return load().qr_factor_ex(m, n, _ptr(A), _ld(A), _ptr(tau), _sched(sched), _stream(stream))


def band_reduce(A, w, tauq, taup, stream=None):
    """Two-sided reduction of the square column-major device matrix A to upper
    band form with bandwidth w in place; tauq, taup (n,) device."""
    n = A.shape[0]
    return load().band_reduce(n, _ptr(A), _ld(A), int(w), _ptr(tauq), _ptr(taup), _stream(stream))


def lu_factor_info():
    info = ctypes.c_int(0)
    rc = load().lu_factor_info(ctypes.byref(info))
    return rc, info.value


def lu_schedule_default(n, prec=LU_FP64):
    s = Schedule()
    rc = load().lu_schedule_default(int(n), int(prec), ctypes.byref(s))
    return rc, (s.b, s.depth, s.panel_cus, s.taper)


def lu_solve(LU, ipiv, B):
    n = LU.shape[0]
    nrhs = 1 if B.dim() == 1 else B.shape[1]
    return load().lu_solve(n, nrhs, _ptr(LU), _ptr(ipiv), _ptr(B))


def lu_solve_ex(LU, ipiv, B, stream=None):
    n = LU.shape[0]
    nrhs = 1 if B.dim() == 1 else B.shape[1]
    return load().lu_solve_ex(n, nrhs, _ptr(LU), _ld(LU), _ptr(ipiv), _ptr(B), _ld(B), _stream(stream))


def lu_solve_noalloc(LU, ipiv, B, stream=None):
    """lu_solve_ex with statically allocated scratch memory (no allocation)."""
    n = LU.shape[0]
    nrhs = 1 if B.dim() == 1 else B.shape[1]
    return load().lu_solve_noalloc(n, nrhs, _ptr(LU), _ld(LU), _ptr(ipiv), _ptr(B), _ld(B), _stream(stream))


def lu_solve_ir(A, B, X, prec=LU_MIXED_FP16, max_iter=10, stream=None):
    """Returns (status, iterations, final HPL residual)."""
    n = A.shape[0]
    nrhs = 1 if B.dim() == 1 else B.shape[1]
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    rc = load().lu_solve_ir(n, nrhs, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(X), _ld(X), int(prec),
                            int(max_iter), ctypes.byref(it), ctypes.byref(res), _stream(stream))
    return rc, it.value, res.value


def lu_selector_load(path):
    """path None: drop the active weights (the fixed default is used)."""
    return load().lu_selector_load(None if path is None else str(path).encode())


def lu_selector_save(path):
    return load().lu_selector_save(str(path).encode())


def lu_selector_predict(n, prec=LU_FP64):
    s = Schedule()
    rc = load().lu_selector_predict(int(n), int(prec), ctypes.byref(s))
    return rc, (s.b, s.depth, s.panel_cus)


def lu_selector_train(X, Y, epochs, lr=1e-2, seed=0):
    """X: float32 (B, 4), Y: int32 (B, 3) numpy arrays. Returns (rc, losses)."""
    import numpy as np
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.int32)
    loss = np.zeros(max(1, int(epochs)), dtype=np.float32)
    rc = load().lu_selector_train(X.ctypes.data, Y.ctypes.data, len(X), int(epochs), float(lr), int(seed),
                                  loss.ctypes.data)
    return rc, loss


def lu_selector_grad(X, Y):
    import numpy as np
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.int32)
    loss = np.zeros(1, dtype=np.float32)
    g = np.zeros(SELECTOR_PARAMS, dtype=np.float32)
    rc = load().lu_selector_grad(X.ctypes.data, Y.ctypes.data, len(X), loss.ctypes.data, g.ctypes.data)
    return rc, float(loss[0]), g


def lu_selector_get_params():
    import numpy as np
    th = np.zeros(SELECTOR_PARAMS, dtype=np.float32)
    rc = load().lu_selector_get_params(th.ctypes.data, SELECTOR_PARAMS)
    return rc, th


def lu_selector_set_params(theta, n_min, n_max):
    import numpy as np
    th = np.ascontiguousarray(theta, dtype=np.float32)
    return load().lu_selector_set_params(th.ctypes.data, len(th), int(n_min), int(n_max))


def lu_release():
    load().lu_release()


def _tasks(arr, rc):
    out = []
    for t in arr[:rc]:
        out.append(dict(kind=t.kind, step=t.step, col_begin=t.col_begin, col_end=t.col_end,
                        stream=t.stream, waits=[t.wait[i] for i in range(t.nwait)], record=t.record))
    return out


def lu_plan_build(n, b, depth, max_tasks=None):
    """Task list of the look-ahead schedule (host only). Returns (rc, list of dicts)."""
    if max_tasks is None:
        N = (n + b - 1) // b if b > 0 else 0
        max_tasks = 8 * N + 16
    arr = (PlanTask * max(1, max_tasks))()
    rc = load().lu_plan_build(int(n), int(b), int(depth), arr, int(max_tasks))
    if rc < 0:
        return rc, []
    return rc, _tasks(arr, rc)


def lu_plan_panels(n, b, taper, prec=LU_FP64, max_starts=None):
    """Panel boundaries [0, ..., n] of a schedule (host only). Returns (rc, list)."""
    if max_starts is None:
        max_starts = n + 2
    arr = (ctypes.c_int * max(1, max_starts))()
    rc = load().lu_plan_panels(int(n), int(b), int(taper), int(prec), arr, int(max_starts))
    if rc < 0:
        return rc, []
    return rc, list(arr[:rc + 1]) if rc > 0 else []


def lu_plan_build_panels(n, starts, depth, max_tasks=None):
    """Task list for explicit panel boundaries (host only). Returns (rc, list of dicts)."""
    N = max(0, len(starts) - 1)
    if max_tasks is None:
        max_tasks = 8 * N + 16
    st = (ctypes.c_int * max(1, len(starts)))(*starts)
    arr = (PlanTask * max(1, max_tasks))()
    rc = load().lu_plan_build_panels(int(n), st, N, int(depth), arr, int(max_tasks))
    if rc < 0:
        return rc, []
    return rc, _tasks(arr, rc)


def lu_plan_build_panels_ex(n, starts, depth, interchanges, max_tasks=None):
    """Task list for explicit panel boundaries, with or without the LU's
    interchange tasks (interchanges: 0 none, 1 one LSWAP per step, 2 one
    deferred LPERM at the end; host only). Returns (rc, list of dicts)."""
    N = max(0, len(starts) - 1)
    if max_tasks is None:
        max_tasks = 8 * N + 16
    st = (ctypes.c_int * max(1, len(starts)))(*starts)
    arr = (PlanTask * max(1, max_tasks))()
    rc = load().lu_plan_build_panels_ex(int(n), st, N, int(depth), int(interchanges), arr, int(max_tasks))
    if rc < 0:
        return rc, []
    return rc, _tasks(arr, rc)


def lu_k_panel(P, ipiv_rel, prec=LU_FP64, wgs=0, d_info=None, stream=None, m=None, w=None):
    m = P.shape[0] if m is None else m
    w = P.shape[1] if w is None else w
    return load().lu_k_panel(int(prec), m, w, _ptr(P), _ld(P), _ptr(ipiv_rel), int(wgs), _ptr(d_info),
                             _stream(stream))


def lu_k_update(L, ipiv_rel, C, prec=LU_FP64, stream=None):
    m, w = L.shape
    return load().lu_k_update(int(prec), m, w, C.shape[1], _ptr(L), _ld(L), _ptr(ipiv_rel), _ptr(C), _ld(C),
                              _stream(stream))


def lu_k_gemm(A, B, C, prec=LU_FP64, stream=None):
    m, k = A.shape
    n = B.shape[1]
    return load().lu_k_gemm(int(prec), m, n, k, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(C), _ld(C),
                            _stream(stream))


def lu_k_laswp(C, ipiv_rel, w, prec=LU_FP64, stream=None):
    m, ncols = C.shape
    return load().lu_k_laswp(int(prec), m, int(w), ncols, _ptr(ipiv_rel), _ptr(C), _ld(C), _stream(stream))


def lu_k_probe_mfma_f64(out, stream=None):
    return load().lu_k_probe_mfma_f64(_ptr(out), _stream(stream))


def lu_k_timing(enable):
    return load().lu_k_timing(int(enable))


def lu_k_timing_read():
    """(rc, summed GEMM ms, summed GEMM flops, launches) of the recorded factorizations."""
    ms = ctypes.c_double(0)
    fl = ctypes.c_double(0)
    n = ctypes.c_int(0)
    rc = load().lu_k_timing_read(ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(n))
    return rc, ms.value, fl.value, n.value


def lu_k_timing_read_ex(kind):
    """(rc, summed ms, summed flops, summed algorithmic bytes, launches) of the
    recorded trailing-GEMM launches of one kind (0 FP64/FP32, 1 FP16/BF16)."""
    ms = ctypes.c_double(0)
    fl = ctypes.c_double(0)
    by = ctypes.c_double(0)
    n = ctypes.c_int(0)
    rc = load().lu_k_timing_read_ex(int(kind), ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by), ctypes.byref(n))
    return rc, ms.value, fl.value, by.value, n.value
