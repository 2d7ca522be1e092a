// C ABI of the look-ahead LU library: argument checks, workspace, schedule
// resolution and the executor that turns the task plan into launches on the
// caller's stream (trailing updates) and the library's panel stream.
//
// Method (paper): the blocked right-looking LU of Sec. 3.5 (RL1-RL3), with
// the row interchanges of LAPACK getrf (Sec. 3.4), reorganised with static
// look-ahead (Sec. 4, Listing 5).  The panel kernel of step j runs on the
// panel stream while the right part of the trailing update of the step before
// runs on the caller's stream; the waits between the two streams come from
// the plan (plan.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "../../include/lu.h"
#include "../../include/lu_kernels.h"
#include "kernels.hpp"
#include "moves.hpp"
#include "plan.hpp"
#include "selector.hpp"
#include "state.hpp"

namespace lu {

namespace {
std::map<int, DeviceState*> g_states;

// optional per-launch timing of the trailing GEMMs: kind 0 = the FP64/FP32
// trailing GEMM, kind 1 = the FP16/BF16 one of the mixed precisions
struct GemmTiming {
    bool on = false;
    std::vector<hipEvent_t> ev;     // start/stop pairs
    std::vector<double> flops, bytes;
    std::vector<int> kind;
    size_t used = 0;                // pairs in use
} g_timing;

int timed_begin(hipStream_t st, int M, int N, int K, hipEvent_t* stop, int kind = 0, double bytes = 0.0) {
    *stop = nullptr;
    if (!g_timing.on) return 0;
    if (g_timing.used * 2 + 2 > g_timing.ev.size()) {
        for (int i = 0; i < 2 * 256; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return LU_ERR_HIP;
            g_timing.ev.push_back(e);
        }
    }
    hipEvent_t start = g_timing.ev[2 * g_timing.used];
    *stop = g_timing.ev[2 * g_timing.used + 1];
    g_timing.flops.resize(g_timing.used + 1);
    g_timing.bytes.resize(g_timing.used + 1);
    g_timing.kind.resize(g_timing.used + 1);
    g_timing.flops[g_timing.used] = 2.0 * M * (double)N * K;
    g_timing.bytes[g_timing.used] = bytes;
    g_timing.kind[g_timing.used] = kind;
    g_timing.used++;
    return hipEventRecord(start, st) == hipSuccess ? 0 : LU_ERR_HIP;
}
constexpr int kEventRing = 1024;
constexpr int kClaimWords = 16 + 2 * 3;   // GEMM: 2 x 8 chunk counters; swap+TRSM and left swaps: 2 each
constexpr int kMaxCand = 256;       // max panel work-groups
constexpr int kNB = 16;             // panel register block width (panel.hip)
}  // namespace

int ensure_events(DeviceState* s, size_t count) {
    // a factorization records each event at most once, so the ring never
    // wraps onto an event that a later task still waits for
    while (s->events.size() < count) {
        hipEvent_t e;
        LU_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        s->events.push_back(e);
    }
    return 0;
}

int ensure(Buffer& b, size_t bytes) {
    if (bytes <= b.bytes && b.ptr) return 0;
    if (b.ptr) {
        if (hipDeviceSynchronize() != hipSuccess) return LU_ERR_HIP;
        hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    if (bytes == 0) return 0;
    if (hipMalloc(&b.ptr, bytes) != hipSuccess) return LU_ERR_NOMEM;
    b.bytes = bytes;
    return 0;
}

void release(Buffer& b) {
    if (b.ptr) hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
}

// XCD of work-groups 0..63 of one launch (out: host int[64]); 0 or LU_ERR_HIP.
int probe_xcds(int* out) {
    int* d = nullptr;
    (void)hipGetLastError();          // a stale error of an earlier call must not fail this check
    if (hipMalloc(&d, 64 * sizeof(int)) != hipSuccess) return LU_ERR_HIP;
    int rc = launch_xcd_probe(d, 64, nullptr);
    if (rc == 0 && hipMemcpy(out, d, 64 * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) rc = LU_ERR_HIP;
    hipFree(d);
    return rc == 0 ? 0 : LU_ERR_HIP;
}

DeviceState* device_state(int* err) {
    *err = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { *err = LU_ERR_HIP; return nullptr; }
    auto it = g_states.find(dev);
    if (it != g_states.end()) return it->second;
    DeviceState* s = new DeviceState();
    s->dev = dev;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) { *err = LU_ERR_HIP; delete s; return nullptr; }
    s->num_cus = prop.multiProcessorCount;
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate_khz <= 0)
        rate_khz = 100000;
    s->spin_limit = (long long)rate_khz * 1000ll * 2;   // 2 seconds
    s->panel_occupancy = 1;
    if (const char* e = std::getenv("LU_PANEL_OCC")) s->panel_occupancy = std::atoi(e) == 2 ? 2 : 1;
    if (const char* e = std::getenv("LU_WIDE_ROWS")) {
        const int v = std::atoi(e);
        if (v > 0) s->wide_rows = v;
    }
    if (const char* e = std::getenv("QR_SPLIT_ROWS")) {
        const int v = std::atoi(e);
        if (v >= 256 && v % 16 == 0) s->qr_split_rows = v;
    }
    if (const char* e = std::getenv("LU_DEBUG_BARRIER_SPIN")) {
        long long v = std::atoll(e);
        if (v > 0) s->spin_limit = v;                    // debug knob: tiny bound forces the timeout path
    }
    // the three streams are created together, so the runtime spreads them over
    // distinct hardware queues whatever streams the caller has made: work on
    // them can then run concurrently (the caller's stream is joined by events)
    if (hipStreamCreateWithFlags(&s->update_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->panel_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->swap_stream, hipStreamNonBlocking) != hipSuccess) {
        *err = LU_ERR_HIP; delete s; return nullptr;
    }
    s->events.resize(kEventRing);
    for (auto& e : s->events)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { *err = LU_ERR_HIP; return nullptr; }
    if (hipMalloc(&s->sync, 8 * sizeof(unsigned)) != hipSuccess) { *err = LU_ERR_NOMEM; return nullptr; }
    if (hipMemset(s->sync, 0, 8 * sizeof(unsigned)) != hipSuccess) { *err = LU_ERR_HIP; return nullptr; }
    if (hipMalloc(&s->info, 4 * sizeof(int)) != hipSuccess) { *err = LU_ERR_NOMEM; return nullptr; }
    if (hipMemset(s->info, 0, 4 * sizeof(int)) != hipSuccess) { *err = LU_ERR_HIP; return nullptr; }
    // the one-XCD panel placement needs the work-groups of a launch dealt
    // round-robin to the 8 XCDs (work-group b on XCD (b + offset) % 8, the
    // offset varying from launch to launch), so that 8 P of them put P on each
    // XCD: probe it once
    if (s->num_cus % 8 == 0) {
        int h[64];
        s->xcd_round_robin = probe_xcds(h) == 0 ? 1 : 0;
        for (int b = 0; b < 64; ++b) s->xcd_round_robin &= ((h[b] - h[0] - b) % 8 + 8) % 8 == 0 ? 1 : 0;
    }
    if (const char* e = std::getenv("LU_PANEL_XCD")) s->panel_one_xcd = std::atoi(e) > 0 ? 1 : 0;
    if (const char* e = std::getenv("LU_ISLAND")) s->island = std::atoi(e) > 0 ? 1 : 0;
    // tagged exchange area of the panel kernel (sized for FP64 and the maximum work-group count)
    if (ensure(s->cand, (size_t)kPanelXchWords * sizeof(unsigned long long))) { *err = LU_ERR_NOMEM; return nullptr; }
    if (hipMemset(s->cand.ptr, 0, s->cand.bytes) != hipSuccess) { *err = LU_ERR_HIP; return nullptr; }
    g_states[dev] = s;
    return s;
}

int begin_factorization(DeviceState* s, hipStream_t stream) {
    const int ring = (int)s->events.size();
    if (ring < 4) return LU_ERR_HIP;
    auto next = [&]() {
        hipEvent_t e = s->events[s->ev_next];
        s->ev_next = (s->ev_next + 1) % ring;
        return e;
    };
    hipEvent_t ev0 = next(), evp = next(), evs = next(), evc = next();
    LU_HIP(hipEventRecord(ev0, stream));
    LU_HIP(hipEventRecord(evp, s->panel_stream));
    LU_HIP(hipEventRecord(evs, s->swap_stream));
    LU_HIP(hipStreamWaitEvent(s->update_stream, ev0, 0));
    LU_HIP(hipStreamWaitEvent(s->update_stream, evp, 0));
    LU_HIP(hipStreamWaitEvent(s->update_stream, evs, 0));
    // error words of both barrier slots (sync[1], sync[3]); the counters are
    // reset by the launches themselves
    if (launch_fill_zero(s->sync + 1, sizeof(unsigned), s->update_stream)) return LU_ERR_HIP;
    if (launch_fill_zero(s->sync + 3, sizeof(unsigned), s->update_stream)) return LU_ERR_HIP;
    LU_HIP(hipEventRecord(evc, s->update_stream));
    LU_HIP(hipStreamWaitEvent(s->panel_stream, evc, 0));
    LU_HIP(hipStreamWaitEvent(s->swap_stream, evc, 0));
    return 0;
}

void release_all() {
    for (auto& kv : g_states) {
        DeviceState* s = kv.second;
        hipSetDevice(s->dev);
        hipDeviceSynchronize();
        for (auto& e : s->events) hipEventDestroy(e);
        if (s->update_stream) hipStreamDestroy(s->update_stream);
        if (s->panel_stream) hipStreamDestroy(s->panel_stream);
        if (s->swap_stream) hipStreamDestroy(s->swap_stream);
        if (s->sync) hipFree(s->sync);
        if (s->info) hipFree(s->info);
        Buffer* bufs[] = {&s->plan_starts, &s->claims, &s->cand, &s->moves, &s->linv, &s->lh, &s->uh, &s->rs, &s->cs, &s->solve_moves, &s->flags,
                          &s->partial, &s->ir_r, &s->ir_x32, &s->ir_a32, &s->ir_a64, &s->ir_norms, &s->ir_ipiv,
                          &s->ir_b, &s->qr_v, &s->qr_vt, &s->qr_t, &s->qr_tt, &s->qr_w, &s->qr_ws, &s->qr_ym, &s->qr_part,
                          &s->band_z, &s->band_v, &s->band_vt, &s->band_t, &s->band_tt, &s->band_w,
                          &s->band_y, &s->band_ws, &s->band_pan};
        for (Buffer* b : bufs) release(*b);
        delete s;
    }
    g_states.clear();
}

int panel_wgs_for(const DeviceState& s, int m, int panel_cus, bool wide) {
    // Rows per work-group: up to 2*threads (the register-resident variants),
    // 4*threads when even kPanelMaxWgs groups would not cover m that way, or
    // when `wide` asks for fewer, fuller groups (a tall FP64 panel that runs
    // beside a long trailing update: its CUs are worth more to the update).
    const int t = panel_threads();
    int need = (m + 2 * t - 1) / (2 * t);
    if (need > kPanelMaxWgs || wide) need = (m + panel_max_rows_per_wg() - 1) / panel_max_rows_per_wg();
    // no more groups than rows / threads: fewer, fuller groups make cheaper barriers
    const int useful = std::max(need, (m + t - 1) / t);
    const int wgs = std::min(std::max(need, std::max(1, panel_cus)), useful);
    if (wgs > kPanelMaxWgs || wgs > s.num_cus) return -1;
    return wgs;
}

namespace {

// ---------------------------------------------------------------- schedule
bool valid_b(int b) { return b == 32 || b == 64 || b == 128 || b == 256 || b == 512; }

int env_int(const char* name, int dflt) {
    const char* e = std::getenv(name);
    if (!e || !*e) return dflt;
    return std::atoi(e);
}

constexpr int kTaperDefault = 1;   // the early-termination taper is on unless asked otherwise

void resolve_schedule(int n, lu_precision_t prec, const lu_schedule_t* req, lu_schedule_t* out) {
    lu_schedule_t s = {256, 1, 16, kTaperDefault};
    lu_schedule_t sel;
    const bool sel_on = selector_enabled() && selector_predict(n, (int)prec, &sel) == 0;
    if (sel_on) { s.b = sel.b; s.depth = sel.depth; s.panel_cus = sel.panel_cus; }
    int e;
    if ((e = env_int("LU_B", 0)) > 0 && valid_b(e)) s.b = e;
    if ((e = env_int("LU_DEPTH", -1)) >= 0 && e <= 2) s.depth = e;
    if ((e = env_int("LU_PANEL_CUS", 0)) > 0 && e <= 256) s.panel_cus = e;
    if ((e = env_int("LU_TAPER", 0)) != 0) s.taper = e > 0 ? 1 : -1;
    if (req) {
        if (req->b > 0) s.b = req->b;
        if (req->depth >= 0 && req->depth <= 2 && (req->b > 0 || req->depth > 0 || req->panel_cus > 0)) {
            // depth 0 is a legal explicit value only when the caller set some field
            s.depth = req->depth;
        }
        if (req->panel_cus > 0) s.panel_cus = req->panel_cus;
        if (req->taper != 0) s.taper = req->taper > 0 ? 1 : -1;
    }
    *out = s;
}

int prec_class(lu_precision_t prec) { return prec == LU_FP64 ? 0 : prec == LU_FP32 ? 1 : 2; }

const DeviceState::Plan* get_plan(DeviceState* s, int n, const lu_schedule_t& sch, lu_precision_t prec) {
    const int taper = sch.taper > 0 ? 1 : 0;
    const long long key = ((long long)n << 20) | ((long long)sch.b << 8) | (sch.depth << 4) | (taper << 2) |
                          prec_class(prec);
    auto it = s->plans.find(key);
    if (it != s->plans.end()) return &it->second;
    if (s->plans.size() > 64) s->plans.clear();
    DeviceState::Plan p;
    p.starts = panel_starts(n, sch.b, taper, prec_class(prec));
    // left interchanges deferred to one final permutation when a column
    // segment fits the permutation kernel, else one LSWAP task per step
    const int swaps = (p.starts.size() >= 3 && n - p.starts[1] <= kLpermMaxRows) ? 2 : 1;
    if (build_plan(n, p.starts, sch.depth, p.tasks, swaps) < 0) return nullptr;
    return &(s->plans[key] = std::move(p));
}

// ---------------------------------------------------------------- executor
struct HalfNone {};


// island: the factorization keeps XCD 0 for its panels (every panel on at
// most num_cus / 8 work-groups of up to 1024 rows, on XCD 0) while the bulk
// update runs on the other XCDs.
template <typename T>
int run_panel(DeviceState* s, T* A, long long lda, int n, int j0, int w, int* ipiv, int* info, int* moves,
              int wgs_req, hipStream_t st, bool island = false) {
    PanelArgs<T> pa;
    const int m = n - j0;
    pa.A = A + j0 + (long long)j0 * lda;
    pa.lda = (int)lda;
    pa.m = m;
    pa.w = w;
    pa.row_base = j0;
    pa.ipiv = ipiv + j0;
    pa.ipiv_rel = nullptr;
    pa.info = info;
    pa.info_col_base = j0;
    pa.moves = moves;
    pa.sync = s->sync + 2 * s->sync_slot;   // [counter, error]
    pa.sync_next = s->sync + 2 * (1 - s->sync_slot);
    s->sync_slot = 1 - s->sync_slot;
    pa.xch = reinterpret_cast<unsigned long long*>(s->cand.ptr);
    // tags: 22 bits of launch number, 10 bits of column (w <= 512); tag 0 is never used
    s->panel_launches = (s->panel_launches + 1) & 0x3fffff;
    if (s->panel_launches == 0) {
        // numbering wrapped: clear words that could still carry a reused tag
        s->panel_launches = 1;
        if (launch_fill_zero(s->cand.ptr, s->cand.bytes, st) != 0) return LU_ERR_HIP;
    }
    pa.tag_base = (unsigned)s->panel_launches << 10;
    pa.spin_limit = s->spin_limit;
    pa.occupancy = s->panel_occupancy;
    // tall FP64 panels (m > wide_rows) use 4*threads rows per group
    const int per_xcd = s->num_cus / 8;
    const bool wide = (sizeof(T) == 8 && m > s->wide_rows) || (island && m > per_xcd * 2 * panel_threads());
    int wgs = panel_wgs_for(*s, m, island ? std::min(wgs_req, per_xcd) : wgs_req, wide);
    if (wgs < 0) return LU_ERR_UNSUPPORTED;
    if (island && wgs > per_xcd) return LU_ERR_UNSUPPORTED;
    pa.one_xcd = ((island || s->panel_one_xcd) && s->xcd_round_robin && wgs <= per_xcd) ? 1 : 0;
    pa.rank = s->sync + 5;                 // cleared right before the launch, on its stream
    if (pa.one_xcd && launch_fill_zero(pa.rank, sizeof(unsigned), st)) return LU_ERR_HIP;
    return launch_panel<T>(pa, wgs, st) == 0 ? 0 : LU_ERR_HIP;
}

template <typename T, typename H>
int execute(DeviceState* s, int n, T* A, long long lda, int* ipiv, int* info, const lu_schedule_t& sch,
            lu_precision_t prec, hipStream_t stream, bool mixed) {
    const DeviceState::Plan* pl = get_plan(s, n, sch, prec);
    if (!pl) return LU_ERR_UNSUPPORTED;
    const std::vector<PlanTask>* plan = &pl->tasks;
    const std::vector<int>& starts = pl->starts;
    const int N = (int)starts.size() - 1;
    int rc;
    if ((rc = ensure(s->moves, (size_t)N * kMovesLen * sizeof(int)))) return rc;
    int* moves = reinterpret_cast<int*>(s->moves.ptr);
    // inverses of each panel's 16x16 diagonal L blocks (one slot per panel)
    constexpr size_t kLinvPer = (size_t)(kMovesMaxW / 16) * 256;
    if ((rc = ensure(s->linv, (size_t)N * kLinvPer * sizeof(T)))) return rc;
    T* linv = reinterpret_cast<T*>(s->linv.ptr);
    // mixed precision operand copies
    H* Lh = nullptr; H* Uh = nullptr; float* rs = nullptr; float* cs = nullptr;
    long long ldh = 0, lduh = 0;
    if (mixed) {
        ldh = ((long long)n + 7) / 8 * 8 + 8;
        lduh = ((long long)n + 7) / 8 * 8 + 8;
        if ((rc = ensure(s->lh, (size_t)n * ldh * sizeof(H)))) return rc;
        if ((rc = ensure(s->uh, (size_t)n * lduh * sizeof(H)))) return rc;
        if ((rc = ensure(s->rs, (size_t)N * n * sizeof(float)))) return rc;
        if ((rc = ensure(s->cs, (size_t)N * n * sizeof(float)))) return rc;
        Lh = reinterpret_cast<H*>(s->lh.ptr);
        Uh = reinterpret_cast<H*>(s->uh.ptr);
        rs = reinterpret_cast<float*>(s->rs.ptr);
        cs = reinterpret_cast<float*>(s->cs.ptr);
    }
    size_t nrec = 0;
    for (const PlanTask& t : *plan) nrec += t.record ? 1 : 0;
    if ((rc = ensure_events(s, nrec + 2 * kPlanStreams + 2))) return rc;
    const int ring = (int)s->events.size();
    // the left interchanges are ordered on the update stream: run beside the
    // panel they slow it down more than they gain
    hipStream_t streams[kPlanStreams] = {s->update_stream, s->panel_stream, s->update_stream};
    // XCD island: with look-ahead, every panel runs on XCD 0 and the kernels of
    // the update stream leave XCD 0 free, so a panel never waits for the CUs
    // of a long trailing update (a panel work-group needs a whole CU)
    const bool island = s->island && sch.depth >= 1 && s->xcd_round_robin &&
                        (long long)n <= (long long)(s->num_cus / 8) * 4 * panel_threads();
    if (island && !s->claims.ptr) {
        if ((rc = ensure(s->claims, kClaimWords * sizeof(unsigned)))) return rc;
        LU_HIP(hipMemset(s->claims.ptr, 0, s->claims.bytes));
    }
    unsigned* claims = reinterpret_cast<unsigned*>(s->claims.ptr);
    // counters of the XCD-0-free launches on the update stream: ping-pong pairs,
    // each launch clears its successor's (the previous user has finished)
    auto gemm_claim = [&]() {
        XcdClaim c;
        c.ctr = claims + 8 * s->claim_par[0];
        c.next = claims + 8 * (1 - s->claim_par[0]);
        c.cus = s->num_cus;
        s->claim_par[0] ^= 1;
        return c;
    };
    auto one_claim = [&](int kind, unsigned** next) {
        unsigned* c = claims + 16 + 2 * kind + s->claim_par[kind];
        *next = claims + 16 + 2 * kind + (1 - s->claim_par[kind]);
        s->claim_par[kind] ^= 1;
        return c;
    };
    // entry join: the library streams start after everything already on `stream`
    // and after every earlier task of their own; the panel barriers' error
    // words are cleared in between, so a time-out of an earlier factorization
    // does not make this one's panels give up at their first wait
    if ((rc = begin_factorization(s, stream))) return rc;
    std::vector<int> ev_of(plan->size(), -1);
    for (size_t ti = 0; ti < plan->size(); ++ti) {
        const PlanTask& t = (*plan)[ti];
        hipStream_t st = streams[t.stream];
        for (int wv = 0; wv < t.nwait; ++wv) {
            const int e = ev_of[t.wait[wv]];
            if (e < 0) return LU_ERR_UNSUPPORTED;
            LU_HIP(hipStreamWaitEvent(st, s->events[e], 0));
        }
        const int k = t.step;
        const int kb = starts[k];
        const int wk = starts[k + 1] - kb;
        int* mv = moves + (size_t)k * kMovesLen;
        if (t.kind == kTaskPanel) {
            if ((rc = run_panel<T>(s, A, lda, n, kb, wk, ipiv, info, mv, sch.panel_cus, st, island))) return rc;
            if (launch_diag_inv<T>(A, lda, kb, wk, linv + (size_t)k * kLinvPer, st)) return LU_ERR_HIP;
            if (mixed && n - kb - wk > 0) {
                if (launch_l21_half<H>(reinterpret_cast<const float*>(A) + (kb + wk) + (long long)kb * lda, lda,
                                       n - kb - wk, wk, Lh + (long long)(kb + wk) * ldh + kb, ldh,
                                       rs + (size_t)k * n + (kb + wk), st))
                    return LU_ERR_HIP;
            }
        } else if (t.kind == kTaskUpdate) {
            SwapTrsmArgs<T, H> sa;
            sa.A = A; sa.lda = lda; sa.r0 = kb; sa.w = wk; sa.moves = mv; sa.m = n - kb;
            sa.c0 = t.col_begin; sa.c1 = t.col_end; sa.linv = linv + (size_t)k * kLinvPer;
            sa.uh = mixed ? Uh + kb : nullptr;
            sa.lduh = lduh;
            sa.cs = mixed ? cs + (size_t)k * n : nullptr;
            const bool skip_t = island && t.stream != 1;     // panel-stream work may use XCD 0
            sa.claim = skip_t ? one_claim(1, &sa.claim_next) : nullptr;
            if (!skip_t) sa.claim_next = nullptr;
            if (launch_swap_trsm<T, H>(sa, st)) return LU_ERR_HIP;
            const int M = n - kb - wk, Nc = t.col_end - t.col_begin;
            if (M > 0) {
                if (mixed) {
                    // algorithmic bytes: FP32 C read and written, the half operands and the scales read once
                    hipEvent_t stop;
                    const double hb = 8.0 * M * (double)Nc + 2.0 * wk * ((double)M + Nc) + 4.0 * ((double)M + Nc);
                    if ((rc = timed_begin(st, M, Nc, wk, &stop, 1, hb))) return rc;
                    if (launch_gemm_half<H>(M, Nc, wk, Lh + (long long)(kb + wk) * ldh + kb, (int)ldh,
                                            Uh + (long long)t.col_begin * lduh + kb, (int)lduh,
                                            rs + (size_t)k * n + (kb + wk), cs + (size_t)k * n + t.col_begin,
                                            reinterpret_cast<float*>(A) + (kb + wk) + (long long)t.col_begin * lda,
                                            (int)lda, st, skip_t ? gemm_claim() : XcdClaim()))
                        return LU_ERR_HIP;
                    if (stop) LU_HIP(hipEventRecord(stop, st));
                } else {
                    hipEvent_t stop;
                    if ((rc = timed_begin(st, M, Nc, wk, &stop))) return rc;
                    if (launch_gemm<T>(M, Nc, wk, A + (kb + wk) + (long long)kb * lda, (int)lda,
                                       A + kb + (long long)t.col_begin * lda, (int)lda,
                                       A + (kb + wk) + (long long)t.col_begin * lda, (int)lda, st,
                                       skip_t ? gemm_claim() : XcdClaim()))
                        return LU_ERR_HIP;
                    if (stop) LU_HIP(hipEventRecord(stop, st));
                }
            }
        } else if (t.kind == kTaskLperm) {
            if ((rc = ensure(s->plan_starts, (N + 1) * sizeof(int)))) return rc;
            int* dst = reinterpret_cast<int*>(s->plan_starts.ptr);
            LU_HIP(hipMemcpyAsync(dst, starts.data(), (N + 1) * sizeof(int), hipMemcpyHostToDevice, st));
            if (launch_lperm<T>(A, lda, n, N, starts.data(), dst, moves, st)) return LU_ERR_HIP;
        } else {
            unsigned* nx = nullptr;
            unsigned* cl = island ? one_claim(2, &nx) : nullptr;
            if (launch_lswap<T>(A, lda, kb, wk, n - kb, mv, t.col_begin, t.col_end, st, cl, nx)) return LU_ERR_HIP;
        }
        if (t.record) {
            const int e = s->ev_next;
            s->ev_next = (s->ev_next + 1) % ring;
            LU_HIP(hipEventRecord(s->events[e], st));
            ev_of[ti] = e;
        }
    }
    // exit join
    for (int u = 0; u < kPlanStreams; ++u) {
        hipEvent_t ev1 = s->events[s->ev_next]; s->ev_next = (s->ev_next + 1) % ring;
        LU_HIP(hipEventRecord(ev1, streams[u]));
        LU_HIP(hipStreamWaitEvent(stream, ev1, 0));
    }
    return 0;
}

int check_sched(const lu_schedule_t* s) {
    if (!s) return 0;
    if (s->b > 0 && !valid_b(s->b)) return -6;
    if (s->depth > 2) return -6;
    if (s->panel_cus > 256) return -6;
    return 0;
}

}  // namespace

int factor_impl(int n, void* A, int lda, lu_precision_t prec, int* ipiv, const lu_schedule_t* sched, int* d_info,
                hipStream_t stream) {
    if (n < 0) return -1;
    if (!A && n > 0) return -2;
    if (lda < std::max(1, n)) return -3;
    if (!ipiv && n > 0) return -4;
    if (prec < LU_FP64 || prec > LU_MIXED_BF16) return -5;
    if (int r = check_sched(sched)) return r;
    if (n == 0) return 0;
    int err;
    DeviceState* s = device_state(&err);
    if (!s) return err;
    lu_schedule_t sch;
    resolve_schedule(n, prec, sched, &sch);
    if (sch.b > n) sch.b = std::max(32, std::min(sch.b, ((n + 31) / 32) * 32));
    int* info = d_info ? d_info : s->info;
    if (!d_info && launch_fill_zero(s->info, sizeof(int), stream)) return LU_ERR_HIP;
    s->last_stream = stream;
    s->last_info = info;
    switch (prec) {
    case LU_FP64:
        return execute<double, _Float16>(s, n, reinterpret_cast<double*>(A), lda, ipiv, info, sch, prec, stream, false);
    case LU_FP32:
        return execute<float, _Float16>(s, n, reinterpret_cast<float*>(A), lda, ipiv, info, sch, prec, stream, false);
    case LU_MIXED_FP16:
        return execute<float, _Float16>(s, n, reinterpret_cast<float*>(A), lda, ipiv, info, sch, prec, stream, true);
    case LU_MIXED_BF16:
        return execute<float, __bf16>(s, n, reinterpret_cast<float*>(A), lda, ipiv, info, sch, prec, stream, true);
    }
    return -5;
}

int schedule_for(int n, lu_precision_t prec, lu_schedule_t* out) {
    resolve_schedule(n, prec, nullptr, out);
    return 0;
}

}  // namespace lu

// ======================================================================= C ABI
extern "C" {

int lu_factor(int n, double* A, int lda, int* ipiv, hipStream_t stream) {
    return lu::factor_impl(n, A, lda, LU_FP64, ipiv, nullptr, nullptr, stream);
}

int lu_factor_ex(int n, void* A, int lda, lu_precision_t prec, int* ipiv, const lu_schedule_t* sched, int* d_info,
                 hipStream_t stream) {
    return lu::factor_impl(n, A, lda, prec, ipiv, sched, d_info, stream);
}

int lu_factor_info(int* info) {
    if (!info) return -1;
    int err;
    lu::DeviceState* s = lu::device_state(&err);
    if (!s) return err;
    LU_HIP(hipStreamSynchronize(s->last_stream));
    LU_HIP(hipStreamSynchronize(s->panel_stream));
    int h = 0;
    unsigned e[4] = {0, 0, 0, 0};
    LU_HIP(hipMemcpy(&h, s->last_info ? s->last_info : s->info, sizeof(int), hipMemcpyDeviceToHost));
    LU_HIP(hipMemcpy(e, s->sync, 4 * sizeof(unsigned), hipMemcpyDeviceToHost));
    *info = h;
    if (e[1] || e[3]) {
        // a barrier timed out: reset the words so later factorizations start clean
        LU_HIP(hipMemset(s->sync, 0, 8 * sizeof(unsigned)));
        return LU_ERR_BARRIER;
    }
    return 0;
}

int lu_schedule_default(int n, lu_precision_t prec, lu_schedule_t* out) {
    if (!out) return -3;
    return lu::schedule_for(n, prec, out);
}

void lu_release(void) { lu::release_all(); }

// ---- per-kernel entry points ------------------------------------------------
int lu_k_panel(lu_precision_t prec, int m, int w, void* P, int ldp, int* ipiv_rel, int wgs, int* d_info,
               hipStream_t stream) {
    if (prec < LU_FP64 || prec > LU_MIXED_BF16) return -1;
    if (m < 1) return -2;
    if (w < 1 || w > m || w > 512) return -3;
    if (!P) return -4;
    if (ldp < m) return -5;
    if (!ipiv_rel) return -6;
    int err;
    lu::DeviceState* s = lu::device_state(&err);
    if (!s) return err;
    int rc = lu::ensure(s->moves, (size_t)lu::kMovesLen * sizeof(int));
    if (rc) return rc;
    lu::PanelArgs<double> pd;
    (void)pd;
    // the panel kernel writes matrix-row pivots; with row_base 0 they are panel-relative
    if (prec == LU_FP64)
        return lu::run_panel<double>(s, reinterpret_cast<double*>(P), ldp, m, 0, w, ipiv_rel, d_info,
                                     reinterpret_cast<int*>(s->moves.ptr), wgs, stream);
    return lu::run_panel<float>(s, reinterpret_cast<float*>(P), ldp, m, 0, w, ipiv_rel, d_info,
                                reinterpret_cast<int*>(s->moves.ptr), wgs, stream);
}

int lu_k_update(lu_precision_t prec, int m, int w, int ncols, const void* L, int ldl, const int* ipiv_rel, void* C,
                int ldc, hipStream_t stream) {
    if (prec < LU_FP64 || prec > LU_MIXED_BF16) return -1;
    if (m < 1) return -2;
    if (w < 1 || w > m || w > 512) return -3;
    if (ncols < 0) return -4;
    if (!L) return -5;
    if (ldl < m) return -6;
    if (!ipiv_rel) return -7;
    if (!C && ncols > 0) return -8;
    if (ldc < m) return -9;
    if (ncols == 0) return 0;
    int err;
    lu::DeviceState* s = lu::device_state(&err);
    if (!s) return err;
    int rc = lu::ensure(s->solve_moves, (size_t)lu::kMovesLen * sizeof(int));
    if (rc) return rc;
    int* mv = reinterpret_cast<int*>(s->solve_moves.ptr);
    if (lu::launch_moves(ipiv_rel, w, m, mv, stream)) return LU_ERR_HIP;
    // The kernels address the panel and the block through one matrix view:
    // they need L and C to share the leading dimension.
    if (ldl != ldc) return LU_ERR_UNSUPPORTED;
    // Treat [L | C] as columns of one matrix starting at column 0 = L: the update
    // kernels take A (matrix base), r0 = 0 and column ranges; C = L + off*ldc.
    const long long off_bytes = reinterpret_cast<const char*>(C) - reinterpret_cast<const char*>(L);
    const size_t esz = prec == LU_FP64 ? 8 : 4;
    if (off_bytes <= 0 || off_bytes % (esz * (long long)ldc) != 0) return LU_ERR_UNSUPPORTED;
    const int c0 = (int)(off_bytes / (esz * (long long)ldc));
    if (c0 < w) return LU_ERR_UNSUPPORTED;
    if ((rc = lu::ensure(s->linv, (size_t)(lu::kMovesMaxW / 16) * 256 * esz))) return rc;
    if (prec == LU_FP64) {
        double* A = const_cast<double*>(reinterpret_cast<const double*>(L));
        double* linv = reinterpret_cast<double*>(s->linv.ptr);
        if (lu::launch_diag_inv<double>(A, ldl, 0, w, linv, stream)) return LU_ERR_HIP;
        lu::SwapTrsmArgs<double, _Float16> sa{A, ldl, 0, w, mv, m, c0, c0 + ncols, linv, nullptr, 0, nullptr, 0};
        if (lu::launch_swap_trsm<double, _Float16>(sa, stream)) return LU_ERR_HIP;
        if (m > w && lu::launch_gemm<double>(m - w, ncols, w, A + w, ldl, A + (long long)c0 * ldl, ldl,
                                             A + w + (long long)c0 * ldl, ldl, stream))
            return LU_ERR_HIP;
    } else {
        float* A = const_cast<float*>(reinterpret_cast<const float*>(L));
        float* linv = reinterpret_cast<float*>(s->linv.ptr);
        if (lu::launch_diag_inv<float>(A, ldl, 0, w, linv, stream)) return LU_ERR_HIP;
        lu::SwapTrsmArgs<float, _Float16> sa{A, ldl, 0, w, mv, m, c0, c0 + ncols, linv, nullptr, 0, nullptr, 0};
        if (lu::launch_swap_trsm<float, _Float16>(sa, stream)) return LU_ERR_HIP;
        if (m > w && lu::launch_gemm<float>(m - w, ncols, w, A + w, ldl, A + (long long)c0 * ldl, ldl,
                                            A + w + (long long)c0 * ldl, ldl, stream))
            return LU_ERR_HIP;
    }
    return 0;
}

int lu_k_gemm(lu_precision_t prec, int m, int n, int k, const void* A, int lda, const void* B, int ldb, void* C,
              int ldc, hipStream_t stream) {
    if (prec < LU_FP64 || prec > LU_MIXED_BF16) return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (k < 0) return -4;
    if (!A && m * k > 0) return -5;
    if (lda < std::max(1, m)) return -6;
    if (!B && k * n > 0) return -7;
    if (ldb < std::max(1, k)) return -8;
    if (!C && m * n > 0) return -9;
    if (ldc < std::max(1, m)) return -10;
    if (m == 0 || n == 0 || k == 0) return 0;
    if (prec == LU_FP64)
        return lu::launch_gemm<double>(m, n, k, (const double*)A, lda, (const double*)B, ldb, (double*)C, ldc,
                                       stream) ? LU_ERR_HIP : 0;
    if (prec == LU_FP32)
        return lu::launch_gemm<float>(m, n, k, (const float*)A, lda, (const float*)B, ldb, (float*)C, ldc,
                                      stream) ? LU_ERR_HIP : 0;
    // mixed: round the operands to half precision with power-of-two scales first
    int err;
    lu::DeviceState* s = lu::device_state(&err);
    if (!s) return err;
    const long long ldh = ((long long)k + 7) / 8 * 8 + 8;
    int rc;
    const size_t hsz = 2;
    if ((rc = lu::ensure(s->lh, (size_t)m * ldh * hsz))) return rc;
    if ((rc = lu::ensure(s->uh, (size_t)n * ldh * hsz))) return rc;
    if ((rc = lu::ensure(s->rs, (size_t)m * sizeof(float)))) return rc;
    if ((rc = lu::ensure(s->cs, (size_t)n * sizeof(float)))) return rc;
    float* rs = (float*)s->rs.ptr;
    float* cs = (float*)s->cs.ptr;
    // A rows -> Lh (row-major, one scale per row); B columns -> Uh (k contiguous, one scale per column)
    if (prec == LU_MIXED_FP16) {
        if (lu::launch_l21_half<_Float16>((const float*)A, lda, m, k, (_Float16*)s->lh.ptr, ldh, rs, stream))
            return LU_ERR_HIP;
        if (lu::launch_cols_half<_Float16>((const float*)B, ldb, k, n, (_Float16*)s->uh.ptr, ldh, cs, stream))
            return LU_ERR_HIP;
        return lu::launch_gemm_half<_Float16>(m, n, k, (_Float16*)s->lh.ptr, (int)ldh, (_Float16*)s->uh.ptr,
                                              (int)ldh, rs, cs, (float*)C, ldc, stream) ? LU_ERR_HIP : 0;
    }
    if (lu::launch_l21_half<__bf16>((const float*)A, lda, m, k, (__bf16*)s->lh.ptr, ldh, rs, stream))
        return LU_ERR_HIP;
    if (lu::launch_cols_half<__bf16>((const float*)B, ldb, k, n, (__bf16*)s->uh.ptr, ldh, cs, stream))
        return LU_ERR_HIP;
    return lu::launch_gemm_half<__bf16>(m, n, k, (__bf16*)s->lh.ptr, (int)ldh, (__bf16*)s->uh.ptr, (int)ldh, rs,
                                        cs, (float*)C, ldc, stream) ? LU_ERR_HIP : 0;
}

int lu_k_laswp(lu_precision_t prec, int m, int w, int ncols, const int* ipiv_rel, void* C, int ldc,
               hipStream_t stream) {
    if (prec < LU_FP64 || prec > LU_MIXED_BF16) return -1;
    if (m < 1) return -2;
    if (w < 1 || w > m || w > 512) return -3;
    if (ncols < 0) return -4;
    if (!ipiv_rel) return -5;
    if (!C && ncols > 0) return -6;
    if (ldc < m) return -7;
    if (ncols == 0) return 0;
    int err;
    lu::DeviceState* s = lu::device_state(&err);
    if (!s) return err;
    int rc = lu::ensure(s->solve_moves, (size_t)lu::kMovesLen * sizeof(int));
    if (rc) return rc;
    int* mv = reinterpret_cast<int*>(s->solve_moves.ptr);
    if (lu::launch_moves(ipiv_rel, w, m, mv, stream)) return LU_ERR_HIP;
    if (prec == LU_FP64)
        return lu::launch_lswap<double>((double*)C, ldc, 0, w, m, mv, 0, ncols, stream) ? LU_ERR_HIP : 0;
    return lu::launch_lswap<float>((float*)C, ldc, 0, w, m, mv, 0, ncols, stream) ? LU_ERR_HIP : 0;
}

int lu_k_timing(int enable) {
    if (enable != 0 && enable != 1) return -1;
    lu::g_timing.on = enable == 1;
    if (enable) lu::g_timing.used = 0;
    return 0;
}

int lu_k_timing_read_ex(int kind, double* ms, double* flops, double* bytes, int* launches) {
    if (kind != 0 && kind != 1) return -1;
    if (!ms) return -2;
    if (!flops) return -3;
    if (!bytes) return -4;
    if (!launches) return -5;
    double t = 0, f = 0, b = 0;
    int cnt = 0;
    for (size_t i = 0; i < lu::g_timing.used; ++i) {
        if (lu::g_timing.kind[i] != kind) continue;
        float e = 0.f;
        LU_HIP(hipEventSynchronize(lu::g_timing.ev[2 * i + 1]));
        LU_HIP(hipEventElapsedTime(&e, lu::g_timing.ev[2 * i], lu::g_timing.ev[2 * i + 1]));
        t += e;
        f += lu::g_timing.flops[i];
        b += lu::g_timing.bytes[i];
        ++cnt;
    }
    *ms = t;
    *flops = f;
    *bytes = b;
    *launches = cnt;
    return 0;
}

int lu_k_timing_read(double* ms, double* flops, int* launches) {
    if (!ms) return -1;
    if (!flops) return -2;
    if (!launches) return -3;
    double b;
    return lu_k_timing_read_ex(0, ms, flops, &b, launches);
}

int lu_k_moves_check(const int* moves, int w, int m, int* out) {
    if (!moves) return -1;
    if (w < 1 || w > lu::kMovesMaxW) return -2;
    if (m < w) return -3;
    if (!out) return -4;
    int k = 0;
    const int nt = lu::moves_top_count(moves, w), ne = lu::moves_extra_count(moves, w);
    for (int s = 0; s < nt; ++s) {
        int d, r;
        if (lu::moves_top(moves, s, w, m, d, r)) { out[2 * k] = d; out[2 * k + 1] = r; ++k; }
    }
    const int ktop = k;
    for (int s = 0; s < ne; ++s) {
        int d, r;
        if (lu::moves_extra(moves, s, w, m, d, r)) { out[2 * k] = d; out[2 * k + 1] = r; ++k; }
    }
    return (ktop << 16) | (k - ktop);
}

int lu_k_xcd_probe(int* out) {
    if (!out) return -1;
    int err;
    lu::DeviceState* s = lu::device_state(&err);
    if (!s) return err;
    int rc = lu::probe_xcds(out);
    if (rc) return rc;
    return s->xcd_round_robin;
}

int lu_k_probe_mfma_f64(double* out, hipStream_t stream) {
    if (!out) return -1;
    return lu::launch_probe_mfma_f64(out, stream) ? LU_ERR_HIP : 0;
}

}  // extern "C"
