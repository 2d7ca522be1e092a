// Panel factorization, RL1 of LU_blk (paper Sec. 3.5): partial-pivoting LU of
// an m x w column block, in place.  This is the "mostly sequential" step that
// the look-ahead overlaps with the trailing update (Sec. 3.6, Sec. 4).
//
// One persistent launch of P work-groups (256 threads each) factors the whole
// panel.  Work-group g owns panel rows [g*R, (g+1)*R), R = 256*RPT; thread t
// holds rows g*R + q*256 + t (q < RPT).  The panel is processed in column
// blocks of NB columns, each held in registers while it is factored:
//
//   for each column j of the block (one device-wide exchange per column):
//     each work-group finds its arg-max of |a| over rows >= the diagonal row d
//     (ties -> smallest row), publishes value, row index and that row's NB
//     block values; the owner of row d publishes row d.  Once every
//     work-group's words have arrived, each picks the same global winner p,
//     swaps rows d and p inside the register block, scales the sub-column by
//     the pivot (true division) and applies the rank-1 update to the
//     remaining block columns.
//   after the block (one device-wide barrier):
//     every work-group applies the block's interchanges to its share of the
//     other panel columns and solves the unit-lower NB x NB system for the
//     block's U rows of those columns to its right (RL2 restricted to the
//     panel); then every work-group updates its own rows of those columns
//     with the block's L (RL3 restricted to the panel).
//
// At the end work-group 0 composes the panel's w interchanges into one
// gather/scatter list (see compose_moves) used by the trailing-update and
// left-swap kernels.
#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace lu {

namespace {

constexpr int kPanelThreads = 256;    // threads per panel work-group
constexpr int kMaxPanelWgs = kPanelMaxWgs;

// Tagged exchange words: every published value is split into 32-bit payloads,
// each paired with the 32-bit tag of the column step in one 64-bit word that is
// written and read with single device-coherent atomic accesses.  A reader
// knows a word is current when its tag matches, so no separate barrier or
// publication order is needed.
template <typename T> struct Wpv;                               // payload words per value
template <> struct Wpv<double> { static constexpr int n = 2; };
template <> struct Wpv<float> { static constexpr int n = 1; };

__device__ __forceinline__ unsigned long long tagged(unsigned tag, unsigned payload) {
    return ((unsigned long long)tag << 32) | payload;
}
template <int S>
__device__ __forceinline__ void put_value(unsigned long long* dst, double v, unsigned tag) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    xstore_s<S>(&dst[0], tagged(tag, (unsigned)(b >> 32)));
    xstore_s<S>(&dst[1], tagged(tag, (unsigned)b));
}
template <int S>
__device__ __forceinline__ void put_value(unsigned long long* dst, float v, unsigned tag) {
    xstore_s<S>(&dst[0], tagged(tag, __float_as_uint(v)));
}
// The same payload words written straight to the work-group's LDS copy
// (xbuf), for a launch of one work-group, which exchanges nothing.
__device__ __forceinline__ void put_lds(unsigned* w, double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    w[0] = (unsigned)(b >> 32);
    w[1] = (unsigned)b;
}
__device__ __forceinline__ void put_lds(unsigned* w, float v) { w[0] = __float_as_uint(v); }
__device__ __forceinline__ double get_value(const unsigned* w, double*) {
    return __longlong_as_double((long long)(((unsigned long long)w[0] << 32) | w[1]));
}
__device__ __forceinline__ float get_value(const unsigned* w, float*) { return __uint_as_float(w[0]); }

// Exchange-area layout (64-bit words), per parity: kMaxPanelWgs candidate slots
// of SW words -- [0] row index, [1, 1+WPV) |value|, then 2*NB row values (WPV
// words each; a step j publishes its register part at positions j..j+NB-1) --
// followed by the diagonal row (2*NB values).
template <typename T, int NB> struct Xch {
    static constexpr int WPV = Wpv<T>::n;
    static constexpr int SW = 1 + WPV + 2 * NB * WPV;        // slot words
    static constexpr int SR = 1 + WPV + NB * WPV;            // slot words read per step
    static constexpr int DW = 2 * NB * WPV;                  // diagonal-row words
    static constexpr int DR = NB * WPV;                      // diagonal-row words read per step
    static constexpr int PAR = kMaxPanelWgs * SW + DW;       // words per parity
};

template <typename X>
__device__ __forceinline__ int nslot_words(int P) { return P * X::SR; }

// Finished block columns of a work-group's rows are kept in LDS when they fit
// (64 KB); otherwise they are read back from the panel in memory.
template <typename T, int NB, int RPT> struct FinCfg {
    static constexpr bool lds = sizeof(T) * NB * RPT * kPanelThreads <= 65536;
    static constexpr int cols = lds ? RPT * kPanelThreads : 1;
};

template <typename T, int NB, int RPT>
struct PanelShared {
    T red_v[2][kPanelThreads / kWave];
    int red_i[2][kPanelThreads / kWave];
    int orslot[2 * (kPanelThreads / kWave)];
    unsigned xbuf[kMaxPanelWgs * Xch<T, NB>::SR + Xch<T, NB>::DR];   // payloads of one step
    T fin[NB][FinCfg<T, NB, RPT>::cols];   // finished block columns of this work-group's rows
    T L[NB][NB + 1];
    T U[kMovesMaxW][NB];          // in-panel update: the block's U rows, transposed
    int piv[kMovesMaxW];          // panel-relative pivot rows of every column so far
    int bmv[1 + 4 * NB];          // block moves: count, (dst, src)...
    int slot_row[2 * NB];         // scratch of the block-move composition
    int content[2 * NB];
    MovesScratch ms;
};

// Composition of a block's nbw (<= NB) interchanges into moves on panel rows,
// computed by one wave with the same formulas as compose_moves (rows relative
// to the block top t0: top rows 0..nbw-1, extra rows >= nbw):
//   L(t) = last t' != t with q[t'] == t;  f(t) = f(L(t)) or t;
//   prev(t) = last t' < t with q[t'] == q[t];
//   top t <- f(t) if q[t]==t, else f(prev(t)) or q[t];  extra e <- f(last t with q[t]==e).
// bmv: [0] number of extra moves, then their (dst, src) pairs as panel rows;
// bmv[1 + 2 NB + t] = source row of top row t (t < nbw).  lt / ft: LDS scratch.
template <int NB>
__device__ __forceinline__ void compose_block_moves(const int* piv, int nbw, int t0, int* bmv, int* lt, int* ft) {
    const int lane = threadIdx.x & (kWave - 1);
    const int q = lane < nbw ? piv[lane] - t0 : -1;
    int Lx = -1, prv = -1;
    bool last = true;
    for (int u = 0; u < nbw; ++u) {            // q of lane u, broadcast from its register
        const int qu = __builtin_amdgcn_readlane(q, u);
        if (u != lane && qu == lane) Lx = u;
        if (qu == q) {
            if (u < lane) prv = u;
            if (u > lane) last = false;
        }
    }
    if (lane < nbw) lt[lane] = Lx;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    if (lane < nbw) {
        int f = lane;
        while (lt[f] >= 0) f = lt[f];
        ft[lane] = f;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    int ex_dst = -1, ex_src = -1;
    if (lane < nbw) {
        const int top_src = (q == lane) ? ft[lane] : (prv >= 0 ? ft[prv] : q);
        bmv[1 + 2 * NB + lane] = t0 + top_src;
        if (q >= nbw && last) { ex_dst = q; ex_src = ft[lane]; }
    }
    // pack the extra moves in lane order
    const bool has_ex = ex_dst >= 0;
    const unsigned long long me = __ballot(has_ex);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (has_ex) {
        const int slot = __popcll(me & below);
        bmv[1 + 2 * slot] = t0 + ex_dst;
        bmv[2 + 2 * slot] = t0 + ex_src;
    }
    if (lane == 0) bmv[0] = __popcll(me);
}

// Interchanges of one block on the other panel columns and, on the columns to
// its right, the unit-lower NB x NB solve for the block's U rows.  One thread
// per column; work-group g of P takes columns t*P + g (thread t), so every CU
// of the panel shares the strided row accesses.  Each thread loads the block's
// top rows from their sources and the extra rows' sources before it stores
// anything, so the column's moves read only old values.
template <typename T, int NB, int S>
__device__ __forceinline__ void block_swap_trsm(T* A, long long lda, int w, int cb, int nbw, int g, int P,
                                                const int* bmv, const T (*L)[NB + 1]) {
    // source indices are clamped to written entries, so no load can use an
    // unset one; the count is the same for every thread (scalar branches)
    const int ne = __builtin_amdgcn_readfirstlane(bmv[0]);
    const int em1 = ne > 0 ? ne - 1 : 0;
    const int* tsrc = bmv + 1 + 2 * NB;
    for (int c = threadIdx.x * P + g; c < w - nbw; c += kPanelThreads * P) {
        const int col = (c < cb) ? c : c + nbw;
        T* colp = A + (long long)col * lda;
        T x[NB], e[NB];
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const T v = cload<S>(colp + tsrc[min(r, nbw - 1)]);
            x[r] = (r < nbw) ? v : T(0);
        }
#pragma unroll
        for (int s = 0; s < NB; ++s) {
            e[s] = T(0);
            if (s < ne) e[s] = cload<S>(colp + bmv[2 + 2 * min(s, em1)]);
        }
        if (col >= cb + nbw) {
            const T* Lf = &L[0][0];
#pragma unroll
            for (int s = 0; s < NB; ++s) {
#pragma unroll
                for (int r = s + 1; r < NB; ++r) x[r] = x[r] - Lf[r * (NB + 1) + s] * x[s];
            }
        }
#pragma unroll
        for (int r = 0; r < NB; ++r)
            if (r < nbw) cstore<S>(colp + cb + r, x[r]);
#pragma unroll
        for (int s = 0; s < NB; ++s)
            if (s < ne) cstore<S>(colp + bmv[1 + 2 * min(s, em1)], e[s]);
    }
}

// In-panel trailing update of one work-group's rows after a block:
// A[i, right0 + c] -= sum_k L[i, cb + k] U[cb + k, right0 + c] for the rows
// i >= right0 of the work-group and c < ncols, on the matrix cores (K = NB = 16,
// four 4-deep MFMA steps per 16 x 16 tile).  Wave v takes the tiles of the
// rows its own lanes hold (row = g*R + q*threads + v*64 + 16 rb + l16); the
// L fragments come from the LDS copy of the finished columns (or from memory
// when that copy does not fit), the U fragments from LDS (staged transposed,
// zero past ncols), and each C tile is loaded, updated and stored once.
template <typename T, int NB, int RPT, int S>
__device__ __forceinline__ void inpanel_update(T* A, long long lda, int g, int m, int cb, int nbw, int right0,
                                               int ncols, const T (*U)[NB],
                                               const T (*fin)[FinCfg<T, NB, RPT>::cols]) {
    static_assert(NB == 16, "one 16-deep k block per update");
    typedef typename Acc<T>::type V4;
    constexpr int R = kPanelThreads * RPT;
    const int tid = threadIdx.x;
    const int wave = tid / kWave, lane = tid % kWave, l16 = lane % 16, lg = lane / 16;
    // -L fragments: lf[q][rb][ks] = -L[row(q, rb, l16)][4 ks + lg]
    T lf[RPT][4][4];
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const int loc = q * kPanelThreads + wave * kWave + rb * 16 + l16;
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int k = 4 * ks + lg;
                T v;
                if constexpr (FinCfg<T, NB, RPT>::lds) v = fin[k][loc];
                else v = cload<S>(A + min(g * R + loc, m - 1) + (long long)(cb + k) * lda);
                lf[q][rb][ks] = (k < nbw) ? -v : T(0);
            }
        }
    const int nct = (ncols + 15) / 16;
    // C tiles of column tile ct
    auto load_c = [&](int ct, V4 (&c)[RPT][4]) {
#pragma unroll
        for (int q = 0; q < RPT; ++q)
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int row = g * R + q * kPanelThreads + wave * kWave + rb * 16 + l16;
                const bool rok = row >= right0 && row < m && ct < nct;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int cc = ct * 16 + Acc<T>::col(lg, r);
                    const bool ok = rok && cc < ncols;
                    const T v = cload<S>(A + (ok ? row : right0) + (long long)(right0 + (ok ? cc : 0)) * lda);
                    c[q][rb][r] = ok ? v : T(0);
                }
            }
    };
    for (int ct = 0; ct < nct; ++ct) {
        V4 cur[RPT][4];
        load_c(ct, cur);
        T uf[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int k = 4 * ks + lg, c = ct * 16 + l16;
            uf[ks] = (c < ncols) ? U[c][k] : T(0);      // U[.][k] is 0 for k >= nbw
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q)
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) cur[q][rb] = mfma(uf[ks], lf[q][rb][ks], cur[q][rb]);
#pragma unroll
        for (int q = 0; q < RPT; ++q)
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int row = g * R + q * kPanelThreads + wave * kWave + rb * 16 + l16;
                const bool rok = row >= right0 && row < m;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = ct * 16 + Acc<T>::col(lg, r);
                    if (rok && c < ncols) cstore<S>(A + row + (long long)(right0 + c) * lda, cur[q][rb][r]);
                }
            }
    }
}

// Column loop of one block, as a shift register: at step j, reg[q][s] holds
// block column j+s of row row_of(q); finished columns go to memory (and to the
// LDS copy `fin`) at once, so every register index is a compile-time constant
// and the loop is not unrolled.
//
// Every access that other work-groups depend on is a relaxed atomic at agent
// scope (see common.hpp).  ONE_XCD places the launch on XCD 0: the grid holds
// 8 work-groups per participant, dealt round-robin to the 8 XCDs; the work-
// groups that find themselves on XCD 0 (hardware register XCC_ID) take a rank
// from a counter (cleared before the launch) and take part, the others return
// at once.  Should fewer than P land there, the first wait runs out and the
// launch reports a barrier time-out.  (Scoping the exchange to one XCD's L2
// instead of the device coherence point was measured: workgroup-scope stores
// and loads between CUs of one XCD did not always see each other.)
template <typename T, int NB, int RPT, int OCC, bool ONE_XCD>
__global__ __launch_bounds__(kPanelThreads) void panel_kernel(PanelArgs<T> a) {
    typedef Xch<T, NB> X;
    constexpr int S = __HIP_MEMORY_SCOPE_AGENT;
    constexpr bool kOneXcd = ONE_XCD;
    __shared__ PanelShared<T, NB, RPT> sh;
    __shared__ int s_rank;
    const int tid = threadIdx.x;
    const int P = kOneXcd ? (int)(gridDim.x >> 3) : (int)gridDim.x;
    int g = (int)blockIdx.x;
    if constexpr (kOneXcd) {
        if (xcd_id() != 0) return;
        if (tid == 0) s_rank = (int)__hip_atomic_fetch_add(a.rank, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        g = s_rank;
        if (g >= P) return;
    }
    const int R = kPanelThreads * RPT;
    const int m = a.m, w = a.w;
    const long long lda = a.lda;
    T* __restrict__ A = a.A;
    unsigned epoch = 0;            // full-barrier count

    if (g == 0 && tid == 0 && a.sync_next) {
        // counter of the next launch's slot (its previous user has finished)
        xstore_s<__HIP_MEMORY_SCOPE_AGENT>(a.sync_next, 0u);
    }
    if (g == 0 && tid == 0 && a.moves) {
        // an empty interchange list until the composition at the end: a panel
        // that gives up at a barrier time-out leaves no stale moves behind
        a.moves[0] = 0;
        a.moves[1] = 0;
    }

    auto row_of = [&](int q) { return g * R + q * kPanelThreads + tid; };
    // finished column t (< NB) of the current block, own row q
    auto fin_get = [&](int t, int q, int cb) -> T {
        if constexpr (FinCfg<T, NB, RPT>::lds) return sh.fin[t][q * kPanelThreads + tid];
        else return cload<S>(A + min(row_of(q), m - 1) + (long long)(cb + t) * lda);
    };
    auto fin_set = [&](int t, int q, T v) {
        if constexpr (FinCfg<T, NB, RPT>::lds) sh.fin[t][q * kPanelThreads + tid] = v;
    };
    // the same for the row of fin column `col` (= q * threads + owner thread)
    auto fin_at = [&](int t, int col, int cb) -> T {
        if constexpr (FinCfg<T, NB, RPT>::lds) return sh.fin[t][col];
        else return cload<S>(A + min(g * R + col, m - 1) + (long long)(cb + t) * lda);
    };
    auto fin_set_at = [&](int t, int col, T v) {
        if constexpr (FinCfg<T, NB, RPT>::lds) sh.fin[t][col] = v;
    };
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;

    for (int cb = 0; cb < w; cb += NB) {
        const int nbw = (w - cb) < NB ? (w - cb) : NB;
        T reg[RPT][NB];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = row_of(q);
            const T* rp = A + min(i, m - 1);        // clamped: unconditional loads, select below
#pragma unroll
            for (int s = 0; s < NB; ++s) {
                const T v = cload<S>(rp + (long long)(cb + min(s, nbw - 1)) * lda);
                reg[q][s] = (i < m && s < nbw) ? v : T(0);
            }
        }

#pragma unroll 1
        for (int j = 0; j < nbw; ++j) {
            const int d = cb + j;
            const unsigned tag = a.tag_base + (unsigned)d;
            unsigned long long* xa = a.xch + (size_t)(d & 1) * X::PAR;     // this step's parity area
            // 1. local arg-max of |a| over rows >= d (current column = slot 0),
            //    wave reduction, then every thread merges the wave results
            T bv = T(-1);
            int bi = 0x7fffffff;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = row_of(q);
                if (i >= d && i < m) argmax_merge(bv, bi, dabs(reg[q][0]), i);
            }
            wave_argmax_all(bv, bi);
            const int rpar = j & 1;                    // red slots alternate between steps
            if ((tid & (kWave - 1)) == 0) { sh.red_v[rpar][tid / kWave] = bv; sh.red_i[rpar][tid / kWave] = bi; }
            lds_barrier();
#pragma unroll
            for (int wv = 0; wv < kPanelThreads / kWave; ++wv) argmax_merge(bv, bi, sh.red_v[rpar][wv], sh.red_i[rpar][wv]);
            // 2. publish: the header of this work-group's candidate (thread 0),
            //    then the candidate's block row and row d, each by the wave that
            //    owns the row: lane t supplies block column t (finished columns
            //    from the LDS copy, the rest read from the owner's registers)
            // A launch of one work-group has no one to exchange with: the same
            // words go straight to its LDS copy (xbuf: the slot's SR words,
            // then row d), and the polling below is skipped.
            const bool solo = P == 1;
            {
                unsigned long long* slot = xa + (size_t)g * X::SW;
                if (tid == 0) {
                    if (solo) {
                        sh.xbuf[0] = (unsigned)bi;
                        put_lds(&sh.xbuf[1], bv);
                    } else {
                        xstore_s<S>(&slot[0], tagged(tag, (unsigned)bi));
                        put_value<S>(&slot[1], bv, tag);
                    }
                }
                if (bi == 0x7fffffff && tid < NB) {    // no candidate here: a zero row completes the slot
                    if (solo) put_lds(&sh.xbuf[1 + X::WPV + tid * X::WPV], T(0));
                    else put_value<S>(&slot[1 + X::WPV + tid * X::WPV], T(0), tag);
                }
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int i = row_of(q);
#pragma unroll
                    for (int which = 0; which < 2; ++which) {
                        const unsigned long long mask = __ballot(which == 0 ? (i == bi) : (i == d));
                        if (mask) {
                            const int ol = __ffsll((long long)mask) - 1;
                            const int col = q * kPanelThreads + wave * kWave + ol;
                            T v = (lane < j) ? fin_at(lane, col, cb) : T(0);
#pragma unroll
                            for (int s = 0; s < NB; ++s) {
                                const T r = lane_t(reg[q][s], ol);
                                if (lane == j + s) v = r;
                            }
                            if (solo) {
                                if (lane < NB) put_lds(&sh.xbuf[(which == 0 ? 1 + X::WPV : X::SR) + lane * X::WPV], v);
                            } else {
                                unsigned long long* dst = which == 0 ? slot + 1 + X::WPV
                                                                     : xa + (size_t)kMaxPanelWgs * X::SW;
                                if (lane < NB) put_value<S>(&dst[lane * X::WPV], v, tag);
                            }
                        }
                    }
                }
            }
            // 3. phase A: every work-group's header and row d, polled until all
            //    words carry this step's tag (bounded wait); one word per thread
            const long long t0 = wall_clock64();
            bool failed = false;
            if (solo) {
                lds_barrier();
            } else {
                // every work-group's slot (header and candidate row) and row d:
                // thread t polls words t, t + threads, ... until all carry this
                // step's tag (bounded wait; thread 0 also watches the error
                // word), then one barrier
                constexpr int MAXW = (kMaxPanelWgs * X::SR + X::DR + kPanelThreads - 1) / kPanelThreads;
                static_assert(MAXW <= 32, "poll mask");
                const int ns = P * X::SR;
                const int total = ns + X::DR;
                int off[MAXW];                              // word offsets in this parity's area
                unsigned pending = 0;
#pragma unroll
                for (int k = 0; k < MAXW; ++k) {
                    const int wi = min(tid + k * kPanelThreads, total - 1);
                    off[k] = wi < ns ? (wi / X::SR) * X::SW + (wi % X::SR) : kMaxPanelWgs * X::SW + (wi - ns);
                    if (tid + k * kPanelThreads < total) pending |= 1u << k;
                }
                int st = 0;
                while (pending) {
                    unsigned long long wv[MAXW];
#pragma unroll
                    for (int k = 0; k < MAXW; ++k) wv[k] = ((pending >> k) & 1u) ? xload_s<S>(xa + off[k]) : 0ull;
                    unsigned errw = 0;
                    if (tid == 0) errw = xload_s<__HIP_MEMORY_SCOPE_AGENT>(a.sync + 1);
#pragma unroll
                    for (int k = 0; k < MAXW; ++k) {
                        if (((pending >> k) & 1u) && (unsigned)(wv[k] >> 32) == tag) {
                            sh.xbuf[tid + k * kPanelThreads] = (unsigned)wv[k];
                            pending &= ~(1u << k);
                        }
                    }
                    if (pending && (errw != 0u || wall_clock64() - t0 > a.spin_limit)) { st = 3; break; }
                }
                st = wg_or(st, sh.orslot, 0, kPanelThreads / kWave);
                failed = (st & 2) != 0;
            }
            if (failed) {
                if (tid == 0) xstore_s<__HIP_MEMORY_SCOPE_AGENT>(a.sync + 1, 1u);
                return;
            }
            // 4. global winner, computed by every wave from the headers (same
            //    decision everywhere: largest magnitude, then smallest row); the
            //    winning row's owner follows from the row distribution
            constexpr int HW = 1 + X::WPV;                 // header words per slot
            const int ns = P * X::SR;                      // xbuf: slots, then row d
            int p, wg;
            {
                T v = T(-1);
                int i = 0x7fffffff;
                if (lane < P) {
                    const unsigned* sw = &sh.xbuf[lane * X::SR];
                    i = (int)sw[0];
                    v = get_value(&sw[1], (T*)nullptr);
                }
                wave_argmax_all(v, i);
                if (i == 0x7fffffff) { p = d; wg = -1; }   // no finite candidate: keep row d
                else { p = i; wg = i / R; }
            }
            // 5. block-row values of row d and of the pivot row (the winning
            //    work-group's candidate row), decoded from xbuf
            auto drow_at = [&](int t) -> T { return get_value(&sh.xbuf[ns + t * X::WPV], (T*)nullptr); };
            auto prow_at = [&](int t) -> T {
                return wg >= 0 ? get_value(&sh.xbuf[wg * X::SR + HW + t * X::WPV], (T*)nullptr) : drow_at(t);
            };
            if (tid == 0) {
                sh.piv[d] = p;
                if (g == 0) {
                    a.ipiv[d] = a.row_base + p;
                    if (a.ipiv_rel) a.ipiv_rel[d] = p;
                }
            }
            if (tid < NB) sh.L[j][tid] = prow_at(tid);     // the finished block row d (for the block step)
            const T piv = prow_at(j);
            if (piv == T(0) && g == 0 && tid == 0 && a.info) atomicCAS(a.info, 0, a.info_col_base + d + 1);
            // 6. rows d and p exchange: the owner's wave writes the block row
            //    to memory and the finished columns to the LDS copy, the owner
            //    lane reloads its register block (columns >= j written to
            //    memory here are rewritten when their own step stores them)
            if (p != d) {
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int i = row_of(q);
#pragma unroll
                    for (int which = 0; which < 2; ++which) {     // 0: row p takes row d; 1: row d takes row p
                        const unsigned long long mask = __ballot(i == (which == 0 ? p : d));
                        if (mask) {
                            const int ol = __ffsll((long long)mask) - 1;
                            const int col = q * kPanelThreads + wave * kWave + ol;
                            const int row = g * R + col;
                            if (lane < nbw) {
                                const T v = which == 0 ? drow_at(lane) : prow_at(lane);
                                cstore<S>(A + row + (long long)(cb + lane) * lda, v);
                                if (lane < j) fin_set_at(lane, col, v);
                            }
                            if (lane == ol) {
#pragma unroll
                                for (int s = 0; s < NB; ++s) {
                                    const int t = min(j + s, NB - 1);
                                    const T v = which == 0 ? drow_at(t) : prow_at(t);
                                    reg[q][s] = (j + s < NB) ? v : T(0);
                                }
                            }
                        }
                    }
                }
            }
            // 7. scale, rank-1 update, store column j, shift
            T pr[NB];
#pragma unroll
            for (int s = 1; s < NB; ++s) {
                const int t = min(j + s, NB - 1);
                pr[s] = (j + s < NB) ? prow_at(t) : T(0);
            }
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = row_of(q);
                if (i > d && i < m) {
                    T l = reg[q][0];
                    if (piv != T(0)) l = l / piv;
                    reg[q][0] = l;
#pragma unroll
                    for (int s = 1; s < NB; ++s) reg[q][s] = reg[q][s] - l * pr[s];
                }
                if (i < m) cstore<S>(A + i + (long long)d * lda, reg[q][0]);
                fin_set(j, q, reg[q][0]);
#pragma unroll
                for (int s = 0; s + 1 < NB; ++s) reg[q][s] = reg[q][s + 1];
                reg[q][NB - 1] = T(0);
            }
            // (the next step's phase A rewrites xbuf only after its first barrier,
            // which every wave reaches after its last read of this step's xbuf)
        }

        const bool more_cols = (w - cb - nbw) > 0 || cb > 0;
        if (more_cols) {
            // every work-group: the block's moves (from its own copy of the
            // pivots) and its share of the columns
            __syncthreads();           // the last step's pivot and block row are in LDS
            // every work-group's rows as its last in-panel update left them: that
            // update completed before its exchange words of this block, which this
            // work-group has read, and the loads below go to the coherence point
            // sh.L rows 0..nbw-1 hold the finished block rows (captured during the
            // column steps); rows past a ragged block's width are cleared
            if (nbw < NB) {
                for (int e = tid; e < NB * NB; e += kPanelThreads) {
                    const int r = e / NB, c = e % NB;
                    if (r >= nbw) sh.L[r][c] = T(0);
                }
            }
            if (tid < kWave) compose_block_moves<NB>(sh.piv + cb, nbw, cb, sh.bmv, sh.slot_row, sh.content);
            __syncthreads();
            block_swap_trsm<T, NB, S>(A, lda, w, cb, nbw, g, P, sh.bmv, sh.L);
            if (grid_barrier_nofence(a.sync, a.sync + 1, ++epoch, a.spin_limit, P)) return;
            // in-panel trailing update of my rows below the block: A[i, right] -= L[i, blk] U[blk, right]
            const int right0 = cb + nbw;
            const int ncols = w - right0;
            if (ncols > 0) {
                for (int e = tid; e < NB * ncols; e += kPanelThreads) {
                    const int s = e % NB, cc = e / NB;
                    sh.U[cc][s] = (s < nbw) ? cload<S>(A + (cb + s) + (long long)(right0 + cc) * lda) : T(0);
                }
                __syncthreads();
                // every row of this work-group lies above right0: nothing to update
                if (g * R + R > right0) inpanel_update<T, NB, RPT, S>(A, lda, g, m, cb, nbw, right0, ncols, sh.U, sh.fin);
                // the next block step of other work-groups reads these rows: they are
                // complete before this work-group's first exchange word of the next block
                wave_mem_drain();
                __syncthreads();
            }
        }
    }

    // compose the whole panel's interchanges for the trailing kernels
    if (g == 0 && a.moves) {
        __syncthreads();
        compose_moves(sh.piv, w, a.moves, sh.ms);
    }
}

}  // namespace

template <typename T>
int launch_panel(const PanelArgs<T>& args, int wgs, hipStream_t stream) {
    constexpr int NB = 16;
    const int m = args.m;
    int rpt = (m + wgs * kPanelThreads - 1) / (wgs * kPanelThreads);
    if (rpt < 1) rpt = 1;
    if (rpt > 4) return -1;   // caller must raise wgs
    dim3 block(kPanelThreads);
    if (args.one_xcd) {
        const dim3 grid(8 * wgs);
        if (rpt == 1) hipLaunchKernelGGL((panel_kernel<T, NB, 1, 1, true>), grid, block, 0, stream, args);
        else if (rpt == 2) hipLaunchKernelGGL((panel_kernel<T, NB, 2, 1, true>), grid, block, 0, stream, args);
        else hipLaunchKernelGGL((panel_kernel<T, NB, 4, 1, true>), grid, block, 0, stream, args);
    } else {
        if (rpt == 1) hipLaunchKernelGGL((panel_kernel<T, NB, 1, 1, false>), dim3(wgs), block, 0, stream, args);
        else if (rpt == 2) hipLaunchKernelGGL((panel_kernel<T, NB, 2, 1, false>), dim3(wgs), block, 0, stream, args);
        else hipLaunchKernelGGL((panel_kernel<T, NB, 4, 1, false>), dim3(wgs), block, 0, stream, args);
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// XCD of each of `wgs` work-groups (out[b] for work-group b): the host checks
// the round-robin deal (work-group b on XCD b % 8) that the one-XCD panel
// placement relies on.
__global__ void xcd_probe_kernel(int* out) {
    if (threadIdx.x == 0) out[blockIdx.x] = xcd_id();
}

int launch_xcd_probe(int* out, int wgs, hipStream_t stream) {
    hipLaunchKernelGGL(xcd_probe_kernel, dim3(wgs), dim3(64), 0, stream, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int panel_max_rows_per_wg() { return kPanelThreads * 4; }
int panel_threads() { return kPanelThreads; }

template int launch_panel<double>(const PanelArgs<double>&, int, hipStream_t);
template int launch_panel<float>(const PanelArgs<float>&, int, hipStream_t);

}  // namespace lu
