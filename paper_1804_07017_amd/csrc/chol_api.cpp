// Cholesky with look-ahead: the LU's task list without interchanges (plan.cpp
// with lswap = false) executed on the same three streams, with the Cholesky
// panel kernel (chol.hip) for PANEL tasks and the lower-triangle symmetric
// update (gemm.hip, syrk_ln_sub) for UPDATE tasks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/chol.h"
#include "kernels.hpp"
#include "plan.hpp"
#include "state.hpp"

namespace lu {

namespace {

bool chol_valid_b(int b) { return b == 32 || b == 64 || b == 128 || b == 256 || b == 512; }

int chol_execute(DeviceState* s, int n, double* A, long long lda, int* info, int b, int depth, int panel_cus,
                 hipStream_t stream) {
    std::vector<int> starts;
    for (int c = 0; c < n; c += b) starts.push_back(c);
    starts.push_back(n);
    const int N = (int)starts.size() - 1;
    std::vector<PlanTask> plan;
    if (build_plan(n, starts, depth, plan, 0) < 0) return LU_ERR_UNSUPPORTED;
    int rc;
    size_t nrec = 0;
    for (const PlanTask& t : plan) nrec += t.record ? 1 : 0;
    if ((rc = ensure_events(s, nrec + 2 * kPlanStreams + 2))) return rc;
    const int ring = (int)s->events.size();
    hipStream_t streams[kPlanStreams] = {s->update_stream, s->panel_stream, s->swap_stream};
    if ((rc = begin_factorization(s, stream))) return rc;
    std::vector<int> ev_of(plan.size(), -1);
    for (size_t ti = 0; ti < plan.size(); ++ti) {
        const PlanTask& t = plan[ti];
        hipStream_t st = streams[t.stream];
        for (int wv = 0; wv < t.nwait; ++wv) {
            const int e = ev_of[t.wait[wv]];
            if (e < 0) return LU_ERR_UNSUPPORTED;
            LU_HIP(hipStreamWaitEvent(st, s->events[e], 0));
        }
        const int k = t.step;
        if (k < 0 || k >= N) return LU_ERR_UNSUPPORTED;
        const int kb = starts[k];
        const int wk = starts[k + 1] - kb;
        if (t.kind == kTaskPanel) {
            CholPanelArgs<double> pa;
            pa.A = A + kb + (long long)kb * lda;
            pa.lda = lda;
            pa.m = n - kb;
            pa.w = wk;
            pa.info = info;
            pa.info_col_base = kb;
            pa.sync = s->sync + 2 * s->sync_slot;
            pa.sync_next = s->sync + 2 * (1 - s->sync_slot);
            s->sync_slot = 1 - s->sync_slot;
            pa.spin_limit = s->spin_limit;
            // one group per 1024 panel rows (four per thread; two once the
            // panel CU share gives enough groups), at least the panel CU share,
            // at most 64 and the CU count (every group must be resident at
            // once).  Fewer groups leave more CUs to the symmetric update
            // running beside the panel: at n = 32768, 32 groups of four rows
            // per thread take 303 ms against 322 ms for 64 groups of two.
            int wgs = std::max((pa.m + 1023) / 1024, std::max(1, panel_cus));
            wgs = std::min(wgs, std::min(64, s->num_cus));
            wgs = std::min(wgs, std::max(1, (pa.m + 255) / 256));
            if ((long long)wgs * 1024 < pa.m) return LU_ERR_UNSUPPORTED;   // > 4 rows per thread
            if (launch_chol_panel<double>(pa, wgs, st)) return LU_ERR_HIP;
        } else if (t.kind == kTaskUpdate) {
            const int c0 = t.col_begin, c1 = t.col_end;
            const double* L = A + c0 + (long long)kb * lda;     // rows c0.. of panel k
            if (launch_syrk_lower<double>(n - c0, c1 - c0, wk, L, (int)lda, L, (int)lda,
                                          A + c0 + (long long)c0 * lda, (int)lda, 0, st))
                return LU_ERR_HIP;
        } else {
            return LU_ERR_UNSUPPORTED;
        }
        if (t.record) {
            const int e = s->ev_next;
            s->ev_next = (s->ev_next + 1) % ring;
            LU_HIP(hipEventRecord(s->events[e], st));
            ev_of[ti] = e;
        }
    }
    for (int u = 0; u < kPlanStreams; ++u) {
        hipEvent_t ev1 = s->events[s->ev_next]; s->ev_next = (s->ev_next + 1) % ring;
        LU_HIP(hipEventRecord(ev1, streams[u]));
        LU_HIP(hipStreamWaitEvent(stream, ev1, 0));
    }
    return 0;
}

}  // namespace

int chol_factor_impl(int n, double* A, int lda, const lu_schedule_t* sched, int* d_info, hipStream_t stream) {
    if (n < 0) return -1;
    if (!A && n > 0) return -2;
    if (lda < std::max(1, n)) return -3;
    int b = 256, depth = 2, panel_cus = 32;
    if (sched) {
        if (sched->b > 0 && !chol_valid_b(sched->b)) return -4;
        if (sched->depth > 2 || sched->panel_cus > 256) return -4;
        if (sched->b > 0) b = sched->b;
        if (sched->depth >= 0 && (sched->b > 0 || sched->depth > 0 || sched->panel_cus > 0)) depth = sched->depth;
        if (sched->panel_cus > 0) panel_cus = sched->panel_cus;
    }
    if (n == 0) return 0;
    int err;
    DeviceState* s = device_state(&err);
    if (!s) return err;
    if ((long long)n > 1024LL * std::min(64, s->num_cus)) return LU_ERR_UNSUPPORTED;
    int* info = d_info ? d_info : s->info;
    if (launch_fill_zero(info, sizeof(int), stream)) return LU_ERR_HIP;
    s->last_stream = stream;
    s->last_info = info;
    return chol_execute(s, n, A, lda, info, b, depth, panel_cus, stream);
}

int chol_solve_impl(int n, int nrhs, const double* L, int lda, double* B, int ldb, hipStream_t stream) {
    int err;
    DeviceState* s = device_state(&err);
    if (!s) return err;
    const int nblk = (n + 63) / 64;
    int rc;
    if (s->flags.bytes < (size_t)nblk * sizeof(int)) {
        if ((rc = ensure(s->flags, (size_t)nblk * sizeof(int)))) return rc;
        LU_HIP(hipMemset(s->flags.ptr, 0, s->flags.bytes));
        s->trsv_epoch = 0;
    }
    int* flags = reinterpret_cast<int*>(s->flags.ptr);
    unsigned* terr = s->sync + 4;                 // the triangular solves' error word
    for (int c = 0; c < nrhs; ++c) {
        if (s->trsv_epoch > 0x3ffffff0) {
            if (launch_fill_zero(s->flags.ptr, s->flags.bytes, stream)) return LU_ERR_HIP;
            s->trsv_epoch = 0;
        }
        const int e1 = ++s->trsv_epoch, e2 = ++s->trsv_epoch;
        if (launch_trsv_chol<double>(L, lda, n, B + (long long)c * ldb, flags, e1, e2, terr, s->spin_limit, stream))
            return LU_ERR_HIP;
    }
    return 0;
}

}  // namespace lu

extern "C" {

int chol_solve(int n, int nrhs, const double* L, int lda, double* B, int ldb, hipStream_t stream) {
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (!L && n > 0) return -3;
    if (lda < std::max(1, n)) return -4;
    if (!B && n > 0 && nrhs > 0) return -5;
    if (ldb < std::max(1, n)) return -6;
    if (n == 0 || nrhs == 0) return 0;
    return lu::chol_solve_impl(n, nrhs, L, lda, B, ldb, stream);
}

int chol_factor(int n, double* A, int lda, hipStream_t stream) {
    return lu::chol_factor_impl(n, A, lda, nullptr, nullptr, stream);
}

int chol_factor_ex(int n, double* A, int lda, const lu_schedule_t* sched, int* d_info, hipStream_t stream) {
    return lu::chol_factor_impl(n, A, lda, sched, d_info, stream);
}

}  // extern "C"
