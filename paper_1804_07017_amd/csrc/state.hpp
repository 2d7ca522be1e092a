// Library-owned per-device state: the panel stream, events, workspace.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <vector>

#include "plan.hpp"

namespace lu {

#define LU_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return LU_ERR_HIP;       \
    } while (0)

struct Buffer {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// Grow-only device allocation; returns 0 or LU_ERR_NOMEM.
int ensure(Buffer& b, size_t bytes);
void release(Buffer& b);

struct DeviceState {
    int dev = -1;
    int num_cus = 0;
    long long spin_limit = 0;          // ~2 s of the device wall clock
    int panel_occupancy = 1;           // panel kernel register budget variant (LU_PANEL_OCC)
    int wide_rows = 20480;             // FP64 panels taller than this use 1024 rows per group (LU_WIDE_ROWS)
    int xcd_round_robin = 0;           // 1: work-group b of a launch runs on XCD b % 8 (probed at set-up)
    int panel_one_xcd = 0;             // LU panels on XCD 0 when they fit its CUs (LU_PANEL_XCD)
    int island = 0;                    // look-ahead with XCD 0 kept for the panels (LU_ISLAND)
    Buffer claims;                     // work counters of the XCD-0-free launches (update stream)
    int claim_par[3] = {0, 0, 0};      // ping-pong parity: GEMM, swap+TRSM, left swaps
    hipStream_t update_stream = nullptr;  // the bulk trailing update
    hipStream_t panel_stream = nullptr;
    hipStream_t swap_stream = nullptr;   // interchanges of finished columns (off the critical path)
    std::vector<hipEvent_t> events;    // ring used for cross-stream dependencies
    int ev_next = 0;

    // panel barrier words: 2 slots x (counter, error); slot alternates per launch
    unsigned* sync = nullptr;
    int sync_slot = 0;
    unsigned panel_launches = 0;       // numbers the panel launches (exchange tags)
    Buffer cand;                       // candidate exchange area of the panel kernel
    Buffer moves;                      // per-panel composed interchanges
    Buffer plan_starts;                // panel boundaries of the running plan (deferred left interchanges)
    Buffer linv;                       // per-panel inverses of the 16x16 diagonal L blocks
    int* info = nullptr;               // library INFO word
    hipStream_t last_stream = nullptr; // stream of the last factorization
    int* last_info = nullptr;

    // mixed precision operand copies
    Buffer lh, uh, rs, cs;
    // QR: explicit V / V^T / T of the last four panels, W and -T^T W per update stream, panel partial sums
    Buffer qr_v, qr_vt, qr_t, qr_tt, qr_w, qr_ws, qr_ym, qr_part;
    Buffer band_z, band_v, band_vt, band_t, band_tt, band_w, band_y, band_ws, band_pan;
    int qr_split_rows = 2048;         // k-slice height of the QR V^T C product (env QR_SPLIT_ROWS)
    // solves / refinement
    Buffer solve_moves, flags, partial, ir_r, ir_x32, ir_a32, ir_a64, ir_norms, ir_ipiv, ir_b;
    int trsv_epoch = 0;

    struct Plan {
        std::vector<int> starts;        // panel boundaries, starts[N] = n
        std::vector<PlanTask> tasks;
    };
    std::map<long long, Plan> plans;
};

DeviceState* device_state(int* err);
// Entry of a factorization on `stream`: the library's update, panel and swap
// streams are ordered after everything already enqueued on `stream` and on
// each other, and the panel barriers' error words are cleared in between
// (so one time-out does not make every later panel give up).  Uses 4 events
// of the ring.
int begin_factorization(DeviceState* s, hipStream_t stream);
int ensure_events(DeviceState* s, size_t count);   // grow the event ring to at least count
void release_all();
int panel_wgs_for(const DeviceState& s, int m, int panel_cus, bool wide = false);

}  // namespace lu
