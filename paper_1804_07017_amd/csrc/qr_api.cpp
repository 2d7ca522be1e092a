// Householder QR with look-ahead: the LU's task list without interchanges
// (plan.cpp with lswap = false) on the library's update and panel streams.
// PANEL(k): the QR panel kernel, then the explicit V, V^T and T^T of the panel
// (ring of four slots: every update of panel k has finished before panel
// k + 4 starts, for any look-ahead depth up to 2).  UPDATE(k, c0, c1) on rows
// kb..m of columns [c0, c1): W = -V^T C as a split-K product over fixed
// 2048-row slices summed in slice order (the slices do not depend on the
// column range, so the look-ahead leaves every element's arithmetic
// unchanged), Ym = -T^T W, C -= V Ym (= C - V T^T V^T C), the products on the
// trailing-update tile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/qr.h"
#include "kernels.hpp"
#include "plan.hpp"
#include "state.hpp"

namespace lu {

namespace {

constexpr int kQrSlots = 4;

bool qr_valid_b(int b) { return b == 32 || b == 64 || b == 128 || b == 256; }

int qr_execute(DeviceState* s, int m, int n, double* A, long long lda, double* tau, int b, int depth,
               hipStream_t stream) {
    std::vector<int> starts;
    for (int c = 0; c < n; c += b) starts.push_back(c);
    starts.push_back(n);
    const int N = (int)starts.size() - 1;
    std::vector<PlanTask> plan;
    if (build_plan(n, starts, depth, plan, 0) < 0) return LU_ERR_UNSUPPORTED;
    int rc;
    const size_t vwords = (size_t)m * b;
    if ((rc = ensure(s->qr_v, kQrSlots * vwords * sizeof(double)))) return rc;
    if ((rc = ensure(s->qr_vt, kQrSlots * vwords * sizeof(double)))) return rc;
    if ((rc = ensure(s->qr_t, (size_t)kQrSlots * b * b * sizeof(double)))) return rc;
    if ((rc = ensure(s->qr_tt, (size_t)kQrSlots * b * b * sizeof(double)))) return rc;
    // V^T C in k-slices of ks rows (fixed per factorization: the slice sums,
    // and so the result, do not depend on how the update is split by columns)
    const int ks = s->qr_split_rows;
    const int max_slices = (m + ks - 1) / ks;
    if (max_slices > 1 && (rc = ensure(s->qr_ws, 2 * (size_t)max_slices * b * n * sizeof(double)))) return rc;
    if ((rc = ensure(s->qr_w, 2 * (size_t)b * n * sizeof(double)))) return rc;
    if ((rc = ensure(s->qr_ym, 2 * (size_t)b * n * sizeof(double)))) return rc;
    if ((rc = ensure(s->qr_part, (size_t)kQrPartWords * sizeof(double)))) return rc;
    double* V = reinterpret_cast<double*>(s->qr_v.ptr);
    double* VT = reinterpret_cast<double*>(s->qr_vt.ptr);
    double* Tb = reinterpret_cast<double*>(s->qr_t.ptr);
    double* TTb = reinterpret_cast<double*>(s->qr_tt.ptr);
    double* WSb = max_slices > 1 ? reinterpret_cast<double*>(s->qr_ws.ptr) : nullptr;
    double* Wb = reinterpret_cast<double*>(s->qr_w.ptr);
    double* Yb = reinterpret_cast<double*>(s->qr_ym.ptr);
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
        const int mk = m - kb;
        const int slot = k % kQrSlots;
        double* Vk = V + slot * vwords;
        double* VTk = VT + slot * vwords;
        double* Tk = Tb + (size_t)slot * b * b;
        double* TTk = TTb + (size_t)slot * b * b;
        if (t.kind == kTaskPanel) {
            QrPanelArgs pa;
            pa.A = A + kb + (long long)kb * lda;
            pa.lda = lda;
            pa.m = mk;
            pa.w = wk;
            pa.tau = tau + kb;
            pa.T = Tk;
            pa.part = reinterpret_cast<double*>(s->qr_part.ptr);
            pa.sync = s->sync + 2 * s->sync_slot;
            pa.sync_next = s->sync + 2 * (1 - s->sync_slot);
            s->sync_slot = 1 - s->sync_slot;
            pa.spin_limit = s->spin_limit;
            // one group per 1024 rows (4 per thread), fixed by the panel height so
            // that the reduction order does not depend on the schedule
            const int wgs = (mk + kQrPanelGroupRows - 1) / kQrPanelGroupRows;
            if (wgs > kQrPanelMaxGroups || wgs > s->num_cus) return LU_ERR_UNSUPPORTED;
            if (launch_qr_panel(pa, wgs, st)) return LU_ERR_HIP;
            if (launch_qr_prep(pa.A, lda, mk, wk, Tk, Vk, VTk, TTk, st)) return LU_ERR_HIP;
        } else if (t.kind == kTaskUpdate) {
            const int c0 = t.col_begin, nc = t.col_end - t.col_begin;
            double* W = Wb + (size_t)(t.stream == 1 ? 1 : 0) * b * n;
            double* Ym = Yb + (size_t)(t.stream == 1 ? 1 : 0) * b * n;
            double* C = A + kb + (long long)c0 * lda;
            const int slices = (mk + ks - 1) / ks;
            const long long cnt = (long long)wk * nc;
            double* Wst = slices > 1 ? WSb + (size_t)(t.stream == 1 ? 1 : 0) * max_slices * b * n : W;
            // W = -V^T C (k-slices summed in slice order), Ym = -T^T W, C -= V Ym
            if (launch_gemm_split<double>(wk, nc, mk, ks, VTk, wk, C, (int)lda, Wst, wk, cnt, st)) return LU_ERR_HIP;
            if (slices > 1 && launch_qr_wsum(Wst, slices, cnt, W, st)) return LU_ERR_HIP;
            if (launch_fill_zero(Ym, (size_t)cnt * sizeof(double), st)) return LU_ERR_HIP;
            if (launch_gemm_hh<double>(wk, nc, wk, TTk, wk, W, wk, Ym, wk, st)) return LU_ERR_HIP;
            if (launch_gemm_hh<double>(mk, nc, wk, Vk, mk, Ym, wk, C, (int)lda, st)) return LU_ERR_HIP;  // C -= V Ym
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

int qr_factor_impl(int m, int n, double* A, int lda, double* tau, const lu_schedule_t* sched, hipStream_t stream) {
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (!A && n > 0) return -3;
    if (lda < std::max(1, m)) return -4;
    if (!tau && n > 0) return -5;
    int b = 128, depth = 2;
    if (sched) {
        if (sched->b > 0 && !qr_valid_b(sched->b)) return -6;
        if (sched->depth > 2 || sched->panel_cus > 256) return -6;
        if (sched->b > 0) b = sched->b;
        if (sched->depth >= 0 && (sched->b > 0 || sched->depth > 0 || sched->panel_cus > 0)) depth = sched->depth;
    }
    if (n == 0) return 0;
    int err;
    DeviceState* s = device_state(&err);
    if (!s) return err;
    if ((long long)m > (long long)kQrPanelGroupRows * std::min(kQrPanelMaxGroups, s->num_cus)) return LU_ERR_UNSUPPORTED;
    // lu_factor_info reports on this factorization: no INFO of its own (0),
    // panel-barrier time-outs through the barrier error words
    if (launch_fill_zero(s->info, sizeof(int), stream)) return LU_ERR_HIP;
    s->last_stream = stream;
    s->last_info = s->info;
    return qr_execute(s, m, n, A, lda, tau, b, depth, stream);
}

}  // namespace lu

extern "C" {

int qr_factor(int m, int n, double* A, int lda, double* tau, hipStream_t stream) {
    return lu::qr_factor_impl(m, n, A, lda, tau, nullptr, stream);
}

int qr_factor_ex(int m, int n, double* A, int lda, double* tau, const lu_schedule_t* sched, hipStream_t stream) {
    return lu::qr_factor_impl(m, n, A, lda, tau, sched, stream);
}

}  // extern "C"
