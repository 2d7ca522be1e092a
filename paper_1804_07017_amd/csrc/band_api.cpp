// Two-sided reduction of a square matrix to upper band form (the first stage
// of a two-stage SVD, the third workload of the paper's evaluation, Sec. 6).
// Iteration k (columns and rows k .. k+kw-1):
//   1. Householder QR of the column panel A[k:n, k:k+kw] (the QR panel kernel),
//      then U_k^T = I - V T^T V^T applied from the left to A[k:n, k+kw:n]:
//      W = -V^T C (k-sliced), Ym = -T^T W, C -= V Ym;
//   2. the row panel A[k:k+w', c0:n] (c0 = k + w, w' = min(kw, n - c0)) is
//      transposed into Z (n - c0 rows), factored by the same panel kernel (its
//      QR is the panel's LQ: L = R^T, the same reflectors and tau) and written
//      back; V_k = I - V T V^T is applied from the right to the rows below,
//      D = A[k+w':n, c0:n]: W2 = -D V (k-sliced), Y2 = -W2 T, D -= Y2 V^T.
// All products run on the trailing-update GEMM kernel.  Look-ahead (Sec. 4
// applied to the two-sided reduction): the right-hand update of iteration k
// writes the next column panel's columns first; that panel is then factored
// on the panel stream while the rest of the update runs on the library's
// update stream, and iteration k + 1 joins it before its left-hand update.
// The caller's stream is joined by events on entry and exit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/band.h"
#include "kernels.hpp"
#include "state.hpp"

namespace lu {

namespace {

constexpr int kBandSub = 128;   // sub-panel width of wide band panels

int band_execute(DeviceState* s, int n, double* A, long long lda, int w, double* tauq, double* taup,
                 hipStream_t caller) {
    int rc;
    const size_t nw = (size_t)n * w;
    const int ks = s->qr_split_rows;
    const int max_slices = (n + ks - 1) / ks;
    // two operand sets: the column panels' (left) and the row panels' (right),
    // so that a column panel factored ahead never overwrites what the running
    // right-hand update reads
    if ((rc = ensure(s->band_z, nw * sizeof(double)))) return rc;
    if ((rc = ensure(s->band_v, 2 * nw * sizeof(double)))) return rc;
    if ((rc = ensure(s->band_vt, 2 * nw * sizeof(double)))) return rc;
    if ((rc = ensure(s->band_t, 2 * (size_t)w * w * sizeof(double)))) return rc;
    if ((rc = ensure(s->band_tt, 2 * (size_t)w * w * sizeof(double)))) return rc;
    if ((rc = ensure(s->band_w, nw * sizeof(double)))) return rc;
    if ((rc = ensure(s->band_y, nw * sizeof(double)))) return rc;
    if (max_slices > 1 && (rc = ensure(s->band_ws, (size_t)max_slices * nw * sizeof(double)))) return rc;
    if ((rc = ensure(s->qr_part, (size_t)kQrPartWords * sizeof(double)))) return rc;
    if ((rc = ensure_events(s, 2 * (size_t)((n + w - 1) / w) + 4))) return rc;
    // wide panels: sub-panel workspace (T, T^T, V of the current sub-panel, V^T
    // of every sub-panel, the Gram and U blocks, the in-panel update's W, Y and
    // k-slices), used only by the stream that factors the panel
    const int nsub = (w + kBandSub - 1) / kBandSub;
    const size_t sub2 = (size_t)kBandSub * kBandSub, nsw = (size_t)n * kBandSub, wsw = (size_t)w * kBandSub;
    const size_t pan_words = 2 * sub2 + nsw + (size_t)nsub * nsw + 4 * wsw + (size_t)std::max(1, max_slices) * wsw;
    if (w > kBandSub && (rc = ensure(s->band_pan, pan_words * sizeof(double)))) return rc;
    double* Tsub = w > kBandSub ? reinterpret_cast<double*>(s->band_pan.ptr) : nullptr;
    double* TTsub = Tsub + sub2;
    double* Vsub = TTsub + sub2;
    double* VTs = Vsub + nsw;                  // [nsub][kBandSub x n], ld kBandSub
    double* Gn = VTs + (size_t)nsub * nsw;     // -(V_i^T V_j) blocks, kBandSub x kBandSub, ld kBandSub
    double* Ub = Gn + wsw;                     // U_i = G_i T_j blocks
    double* Wpn = Ub + wsw;                    // in-panel update W, Y
    double* Ypn = Wpn + wsw;
    double* WSpn = Ypn + wsw;                  // k-slices of the panel's own products
    struct Ops { double *Vw, *VT, *T, *TT; };
    Ops L{reinterpret_cast<double*>(s->band_v.ptr), reinterpret_cast<double*>(s->band_vt.ptr),
          reinterpret_cast<double*>(s->band_t.ptr), reinterpret_cast<double*>(s->band_tt.ptr)};
    Ops R{L.Vw + nw, L.VT + nw, L.T + (size_t)w * w, L.TT + (size_t)w * w};
    double* Z = reinterpret_cast<double*>(s->band_z.ptr);
    double* W = reinterpret_cast<double*>(s->band_w.ptr);
    double* Y = reinterpret_cast<double*>(s->band_y.ptr);
    double* WS = max_slices > 1 ? reinterpret_cast<double*>(s->band_ws.ptr) : nullptr;
    const int ring = (int)s->events.size();
    auto next_event = [&]() { hipEvent_t e = s->events[s->ev_next]; s->ev_next = (s->ev_next + 1) % ring; return e; };

    // one panel factorization (m x pw at P, leading dimension ld) into o / tau on stream q
    auto panel = [&](double* P, long long ld, int m, int pw, double* tau, const Ops& o, hipStream_t q) -> int {
        QrPanelArgs pa;
        pa.A = P;
        pa.lda = ld;
        pa.m = m;
        pa.w = pw;
        pa.tau = tau;
        pa.T = o.T;
        pa.part = reinterpret_cast<double*>(s->qr_part.ptr);
        pa.sync = s->sync + 2 * s->sync_slot;
        pa.sync_next = s->sync + 2 * (1 - s->sync_slot);
        s->sync_slot = 1 - s->sync_slot;
        pa.spin_limit = s->spin_limit;
        const int wgs = (m + kQrPanelGroupRows - 1) / kQrPanelGroupRows;
        if (wgs > kQrPanelMaxGroups || wgs > s->num_cus) return LU_ERR_UNSUPPORTED;
        // T's strictly lower part stays zero: the right-hand update multiplies by T itself
        if (launch_fill_zero(o.T, (size_t)pw * pw * sizeof(double), q)) return LU_ERR_HIP;
        if (launch_qr_panel(pa, wgs, q)) return LU_ERR_HIP;
        if (launch_qr_prep(P, ld, m, pw, o.T, o.Vw, o.VT, o.TT, q)) return LU_ERR_HIP;
        return 0;
    };

    // a panel wider than kBandSub: sub-panels of kBandSub columns, each factored
    // by the panel kernel and applied to the panel's columns right of it as a
    // block reflector; T is assembled blockwise, T[0:j0, j] = -T[0:j0, 0:j0]
    // (V[:, 0:j0]^T V_j) T_j, so the panel's (V, T) is that of the single-launch
    // panel up to rounding, at the cost of three narrow panels instead of one
    // wide one (the panel kernel's blocked work grows with the square of the width)
    auto panel_wide = [&](double* P, long long ld, int m, int pw, double* tau, const Ops& o, hipStream_t q) -> int {
        if (pw <= kBandSub) return panel(P, ld, m, pw, tau, o, q);
        if (launch_fill_zero(o.T, (size_t)pw * pw * sizeof(double), q)) return LU_ERR_HIP;
        for (int j0 = 0, i = 0; j0 < pw; j0 += kBandSub, ++i) {
            const int jw = std::min(kBandSub, pw - j0);
            const int mj = m - j0;
            double* Pj = P + j0 + (long long)j0 * ld;
            double* VTi = VTs + (size_t)i * nsw;
            // the sub-panel: reflectors and T_j, explicit V_j, V_j^T, T_j^T
            QrPanelArgs pa;
            pa.A = Pj;
            pa.lda = ld;
            pa.m = mj;
            pa.w = jw;
            pa.tau = tau + j0;
            pa.T = Tsub;
            pa.part = reinterpret_cast<double*>(s->qr_part.ptr);
            pa.sync = s->sync + 2 * s->sync_slot;
            pa.sync_next = s->sync + 2 * (1 - s->sync_slot);
            s->sync_slot = 1 - s->sync_slot;
            pa.spin_limit = s->spin_limit;
            const int wgs = (mj + kQrPanelGroupRows - 1) / kQrPanelGroupRows;
            if (wgs > kQrPanelMaxGroups || wgs > s->num_cus) return LU_ERR_UNSUPPORTED;
            if (launch_fill_zero(Tsub, (size_t)jw * jw * sizeof(double), q)) return LU_ERR_HIP;
            if (launch_qr_panel(pa, wgs, q)) return LU_ERR_HIP;
            if (launch_qr_prep(Pj, ld, mj, jw, Tsub, Vsub, VTi, TTsub, q)) return LU_ERR_HIP;
            if (launch_copy_f64(Tsub, jw, o.T + j0 + (long long)j0 * pw, pw, jw, jw, q)) return LU_ERR_HIP;
            const int slices = (mj + ks - 1) / ks;
            // T's block above T_j, one earlier sub-panel (rows of T) at a time
            for (int ip = 0; ip < i; ++ip) {
                const int off = j0 - ip * kBandSub;    // rows of sub-panel ip's V^T before row j0
                const double* VTp = VTs + (size_t)ip * nsw + (size_t)off * kBandSub;
                const long long cnt = (long long)kBandSub * jw;
                double* Gi = Gn + (size_t)ip * kBandSub * jw;
                double* Wst = slices > 1 ? WSpn : Gi;
                if (launch_gemm_split<double>(kBandSub, jw, mj, ks, VTp, kBandSub, Vsub, mj, Wst, kBandSub, cnt, q))
                    return LU_ERR_HIP;                                            // -V_ip^T V_j
                if (slices > 1 && launch_qr_wsum(Wst, slices, cnt, Gi, q)) return LU_ERR_HIP;
                double* Ui = Ub + (size_t)ip * kBandSub * jw;
                if (launch_fill_zero(Ui, (size_t)cnt * sizeof(double), q)) return LU_ERR_HIP;
                if (launch_gemm_hh<double>(kBandSub, jw, jw, Gi, kBandSub, Tsub, jw, Ui, kBandSub, q))
                    return LU_ERR_HIP;                                            // U = G T_j
            }
            for (int ip = 0; ip < i; ++ip)                                        // T[0:j0, j] -= T[0:j0, ip] U_ip
                if (launch_gemm_hh<double>(j0, jw, kBandSub, o.T + (long long)ip * kBandSub * pw, pw,
                                           Ub + (size_t)ip * kBandSub * jw, kBandSub, o.T + (long long)j0 * pw, pw,
                                           q)) return LU_ERR_HIP;
            // the panel's columns right of the sub-panel: C -= V_j (T_j^T (V_j^T C))
            const int ncp = pw - j0 - jw;
            if (ncp > 0) {
                double* C = Pj + (long long)jw * ld;
                const long long cnt = (long long)jw * ncp;
                double* Wst = slices > 1 ? WSpn : Wpn;
                if (launch_gemm_split<double>(jw, ncp, mj, ks, VTi, jw, C, (int)ld, Wst, jw, cnt, q)) return LU_ERR_HIP;
                if (slices > 1 && launch_qr_wsum(Wst, slices, cnt, Wpn, q)) return LU_ERR_HIP;
                if (launch_fill_zero(Ypn, (size_t)cnt * sizeof(double), q)) return LU_ERR_HIP;
                if (launch_gemm_hh<double>(jw, ncp, jw, TTsub, jw, Wpn, jw, Ypn, jw, q)) return LU_ERR_HIP;
                if (launch_gemm_hh<double>(mj, ncp, jw, Vsub, mj, Ypn, jw, C, (int)ld, q)) return LU_ERR_HIP;
            }
        }
        if (launch_qr_prep(P, ld, m, pw, o.T, o.Vw, o.VT, o.TT, q)) return LU_ERR_HIP;
        return 0;
    };

    // look-ahead: the column panel of the next iteration is factored on the
    // panel stream once the right-hand update has written its columns, while
    // the rest of that update runs on the update stream
    hipStream_t ps = s->panel_stream;
    hipStream_t st = s->update_stream;
    hipEvent_t ev0 = next_event();
    LU_HIP(hipEventRecord(ev0, caller));
    LU_HIP(hipStreamWaitEvent(ps, ev0, 0));
    LU_HIP(hipStreamWaitEvent(st, ev0, 0));
    if ((rc = panel_wide(A, lda, n, std::min(w, n), tauq, L, st))) return rc;
    hipEvent_t pending = nullptr;              // the column panel factored ahead, not yet joined
    for (int k = 0; k < n; k += w) {
        const int kw = std::min(w, n - k);
        const int mk = n - k;
        if (pending) {
            LU_HIP(hipStreamWaitEvent(st, pending, 0));
            pending = nullptr;
        }
        // 1. the left-hand update of the columns right of the column panel
        const int nc = n - k - kw;
        if (nc > 0) {
            double* C = A + k + (long long)(k + kw) * lda;
            const long long cnt = (long long)kw * nc;
            const int slices = (mk + ks - 1) / ks;
            double* Wst = slices > 1 ? WS : W;
            if (launch_gemm_split<double>(kw, nc, mk, ks, L.VT, kw, C, (int)lda, Wst, kw, cnt, st)) return LU_ERR_HIP;
            if (slices > 1 && launch_qr_wsum(Wst, slices, cnt, W, st)) return LU_ERR_HIP;
            if (launch_fill_zero(Y, (size_t)cnt * sizeof(double), st)) return LU_ERR_HIP;
            if (launch_gemm_hh<double>(kw, nc, kw, L.TT, kw, W, kw, Y, kw, st)) return LU_ERR_HIP;
            if (launch_gemm_hh<double>(mk, nc, kw, L.Vw, mk, Y, kw, C, (int)lda, st)) return LU_ERR_HIP;
        }
        // 2. row panel (as the QR of its transpose) and the right-hand update
        const int c0 = k + w;
        if (c0 >= n) continue;
        const int np = n - c0;
        const int wp = std::min(kw, np);
        double* Rp = A + k + (long long)c0 * lda;
        if (launch_transpose_f64(Rp, lda, wp, np, Z, np, st)) return LU_ERR_HIP;
        if ((rc = panel_wide(Z, np, np, wp, taup + k, R, st))) return rc;
        if (launch_transpose_f64(Z, np, np, wp, Rp, lda, st)) return LU_ERR_HIP;
        const int md = n - k - wp;
        const int kn = std::min(w, n - c0);    // width of the next column panel (its columns start at c0)
        if (md > 0) {
            double* D = A + (k + wp) + (long long)c0 * lda;
            const long long cnt = (long long)md * wp;
            const int slices = (np + ks - 1) / ks;
            double* Wst = slices > 1 ? WS : W;
            if (launch_gemm_split<double>(md, wp, np, ks, D, (int)lda, R.Vw, np, Wst, md, cnt, st)) return LU_ERR_HIP;
            if (slices > 1 && launch_qr_wsum(Wst, slices, cnt, W, st)) return LU_ERR_HIP;
            if (launch_fill_zero(Y, (size_t)cnt * sizeof(double), st)) return LU_ERR_HIP;
            if (launch_gemm_hh<double>(md, wp, wp, W, md, R.T, wp, Y, md, st)) return LU_ERR_HIP;       // Y2 = -W2 T
            // D -= Y2 V^T: the next column panel's columns first (the same
            // per-element operations as one product over all columns)
            if (launch_gemm_hh<double>(md, kn, wp, Y, md, R.VT, wp, D, (int)lda, st)) return LU_ERR_HIP;
        }
        // the next column panel ahead, on the panel stream
        {
            hipEvent_t ready = next_event();
            LU_HIP(hipEventRecord(ready, st));
            LU_HIP(hipStreamWaitEvent(ps, ready, 0));
            const int k1 = k + w;
            if ((rc = panel_wide(A + k1 + (long long)k1 * lda, lda, n - k1, kn, tauq + k1, L, ps))) return rc;
            pending = next_event();
            LU_HIP(hipEventRecord(pending, ps));
        }
        if (md > 0 && np > kn) {
            double* D = A + (k + wp) + (long long)c0 * lda;
            if (launch_gemm_hh<double>(md, np - kn, wp, Y, md, R.VT + (size_t)kn * wp, wp, D + (long long)kn * lda,
                                    (int)lda, st)) return LU_ERR_HIP;
        }
    }
    if (pending) LU_HIP(hipStreamWaitEvent(st, pending, 0));
    hipEvent_t done = next_event();
    LU_HIP(hipEventRecord(done, st));
    LU_HIP(hipStreamWaitEvent(caller, done, 0));
    return 0;
}

}  // namespace

int band_reduce_impl(int n, double* A, int lda, int w, double* tauq, double* taup, hipStream_t stream) {
    if (n < 0) return -1;
    if (!A && n > 0) return -2;
    if (lda < std::max(1, n)) return -3;
    if (w < 1 || w > kQrMaxPanelW) return -4;
    if (!tauq && n > 0) return -5;
    if (!taup && n > 0) return -6;
    if (n == 0) return 0;
    int err;
    DeviceState* s = device_state(&err);
    if (!s) return err;
    if ((long long)n > (long long)kQrPanelGroupRows * std::min(kQrPanelMaxGroups, s->num_cus)) return LU_ERR_UNSUPPORTED;
    if (launch_fill_zero(s->info, sizeof(int), stream)) return LU_ERR_HIP;
    if (launch_fill_zero(taup, (size_t)n * sizeof(double), stream)) return LU_ERR_HIP;
    s->last_stream = stream;
    s->last_info = s->info;
    return band_execute(s, n, A, lda, w, tauq, taup, stream);
}

}  // namespace lu

extern "C" {

int band_reduce(int n, double* A, int lda, int w, double* tauq, double* taup, hipStream_t stream) {
    return lu::band_reduce_impl(n, A, lda, w, tauq, taup, stream);
}

}  // extern "C"
