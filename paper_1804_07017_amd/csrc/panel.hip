// Panel factorization, RL1 of LU_blk (paper Sec. 3.5): partial-pivoting LU of
// an m x w column block, in place.  This is the "mostly sequential" step that
// the look-ahead overlaps with the trailing update (Sec. 3.6, Sec. 4).
//
// One persistent launch of P work-groups (256 threads each) factors the whole
// panel.  Work-group g owns panel rows [g*R, (g+1)*R), R = 256*RPT; thread t
// holds rows g*R + q*256 + t (q < RPT).  The panel is processed in column
// blocks of NB columns, each held in registers while it is factored:
//
//   for each column j of the block (one device-wide barrier per column):
//     each work-group finds its arg-max of |a| over rows >= the diagonal row d
//     (ties -> smallest row), publishes value, row index and that row's NB
//     block values; the owner of row d publishes row d.  After the barrier
//     every work-group picks the same global winner p, swaps rows d and p
//     inside the register block, scales the sub-column by the pivot (true
//     division) and applies the rank-1 update to the remaining block columns.
//   after the block (one more barrier):
//     the work-group owning the block's diagonal rows applies the block's
//     interchanges to the other panel columns and solves the unit-lower
//     NB x NB system for the block's U rows of the columns to its right
//     (RL2 restricted to the panel); then every work-group updates its own
//     rows of those columns with the block's L (RL3 restricted to the panel).
//
// At the end work-group 0 composes the panel's w interchanges into one
// gather/scatter list (see compose_moves) used by the trailing-update and
// left-swap kernels.
#include "common.hpp"
#include "kernels.hpp"

namespace lu {

namespace {

constexpr int kPanelThreads = 256;    // threads per panel work-group
constexpr int kMaxPanelWgs = kPanelMaxWgs;
constexpr int kUChunk = 8;    // right-hand columns per pipelined pass of the in-panel update

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
__device__ __forceinline__ void put_value(unsigned long long* dst, double v, unsigned tag) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    xstore(&dst[0], tagged(tag, (unsigned)(b >> 32)));
    xstore(&dst[1], tagged(tag, (unsigned)b));
}
__device__ __forceinline__ void put_value(unsigned long long* dst, float v, unsigned tag) {
    xstore(&dst[0], tagged(tag, __float_as_uint(v)));
}
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
    T red_v[kPanelThreads / kWave];
    int red_i[kPanelThreads / kWave];
    int win_i;
    int win_g;
    T drow[2 * NB];               // row d of the block, zero padded
    T prow[2 * NB];               // pivot row of the block (block column order), zero padded;
                                  // must follow drow directly (addressed as drow + 2*NB)
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
// bmv: [0] count, then (dst, src) pairs as panel rows.  lt / ft: LDS scratch.
template <int NB>
__device__ __forceinline__ void compose_block_moves(const int* piv, int nbw, int t0, int* bmv, int* lt, int* ft) {
    const int lane = threadIdx.x & (kWave - 1);
    const int q = lane < nbw ? piv[lane] - t0 : -1;
    if (lane < nbw) {
        int L = -1;
        for (int u = 0; u < nbw; ++u)
            if (u != lane && piv[u] - t0 == lane) L = u;
        lt[lane] = L;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    if (lane < nbw) {
        int f = lane;
        while (lt[f] >= 0) f = lt[f];
        ft[lane] = f;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    int top_src = -1, ex_dst = -1, ex_src = -1;
    if (lane < nbw) {
        int prv = -1;
        bool last = true;
        for (int u = 0; u < nbw; ++u) {
            const int qu = piv[u] - t0;
            if (qu == q) {
                if (u < lane) prv = u;
                if (u > lane) last = false;
            }
        }
        top_src = (q == lane) ? ft[lane] : (prv >= 0 ? ft[prv] : q);
        if (q >= nbw && last) { ex_dst = q; ex_src = ft[lane]; }
    }
    // pack the changed moves: lane order, top moves then extra moves
    const bool has_top = lane < nbw && top_src != lane;
    const bool has_ex = ex_dst >= 0;
    const unsigned long long mt = __ballot(has_top), me = __ballot(has_ex);
    const int nt = __popcll(mt);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (has_top) {
        const int slot = __popcll(mt & below);
        bmv[1 + 2 * slot] = t0 + lane;
        bmv[2 + 2 * slot] = t0 + top_src;
    }
    if (has_ex) {
        const int slot = nt + __popcll(me & below);
        bmv[1 + 2 * slot] = t0 + ex_dst;
        bmv[2 + 2 * slot] = t0 + ex_src;
    }
    if (lane == 0) bmv[0] = nt + __popcll(me);
}

// Interchanges of one block on the other panel columns and, on the columns to
// its right, the unit-lower NB x NB solve for the block's U rows.  One thread
// per column.
template <typename T, int NB>
__device__ __forceinline__ void block_swap_trsm(T* A, long long lda, int w, int cb, int nbw,
                                                const int* bmv, const T (*L)[NB + 1]) {
    // Indices are clamped instead of guarded: every load and store is
    // unconditional (surplus lanes repeat the last move / row with its own
    // value), which keeps the code free of per-element branches.
    const int cnt = bmv[0];
    const int cm1 = cnt > 0 ? cnt - 1 : 0;
    for (int c = threadIdx.x; c < w - nbw; c += kPanelThreads) {
        const int col = (c < cb) ? c : c + nbw;
        T* colp = A + (long long)col * lda;
        if (cnt > 0) {
            T v[2 * NB];
#pragma unroll
            for (int s = 0; s < 2 * NB; ++s) v[s] = colp[bmv[2 + 2 * min(s, cm1)]];
#pragma unroll
            for (int s = 0; s < 2 * NB; ++s) colp[bmv[1 + 2 * min(s, cm1)]] = v[s];   // v[s] == v[cm1] for s > cm1
        }
        if (col >= cb + nbw) {
            const T* Lf = &L[0][0];
            T x[NB];
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const T v = colp[cb + min(r, nbw - 1)];
                x[r] = (r < nbw) ? v : T(0);
            }
#pragma unroll
            for (int s = 0; s < NB; ++s) {
#pragma unroll
                for (int r = s + 1; r < NB; ++r) x[r] = x[r] - Lf[r * (NB + 1) + s] * x[s];
            }
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                T xr = x[0];
#pragma unroll
                for (int k = 1; k < NB; ++k) xr = (min(r, nbw - 1) == k) ? x[k] : xr;
                colp[cb + min(r, nbw - 1)] = xr;
            }
        }
    }
}

// Row i of the in-panel trailing update for one chunk of right-hand columns:
// A[i, c0:c0+nc] -= L[i, cb:cb+nbw] U[cb:cb+nbw, c0:c0+nc], U staged in LDS
// (U is staged transposed).
template <typename T, int NB, int RPT>
__device__ __forceinline__ void inpanel_update(T* A, long long lda, const int* rows, int cb, int nbw, int right0,
                                               int ncols, const T (*U)[NB], const T (*fin)[FinCfg<T, NB, RPT>::cols]) {
    // All of the thread's rows (rows[q] < 0: none) are updated together, a
    // chunk of kUChunk columns at a time, with the next chunk's loads in flight
    // while the current one is computed and stored.  Addresses are clamped into
    // the valid range so that every load is unconditional.
    bool act[RPT];
    const T* rp[RPT];
    T l[RPT][NB];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        act[q] = rows[q] >= 0;
        rp[q] = A + (act[q] ? rows[q] : 0);
#pragma unroll
        for (int s = 0; s < NB; ++s) {
            T v;
            if constexpr (FinCfg<T, NB, RPT>::lds) v = fin[s][q * kPanelThreads + threadIdx.x];
            else v = rp[q][(long long)(cb + min(s, nbw - 1)) * lda];
            l[q][s] = (s < nbw) ? v : T(0);
        }
    }
    T x[RPT][kUChunk], y[RPT][kUChunk];
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int cc = 0; cc < kUChunk; ++cc) x[q][cc] = rp[q][(long long)(right0 + min(cc, ncols - 1)) * lda];
    for (int c0 = 0; c0 < ncols; c0 += kUChunk) {
        const int nxt = c0 + kUChunk;
#pragma unroll
        for (int q = 0; q < RPT; ++q)
#pragma unroll
            for (int cc = 0; cc < kUChunk; ++cc) y[q][cc] = rp[q][(long long)(right0 + min(nxt + cc, ncols - 1)) * lda];
#pragma unroll
        for (int cc = 0; cc < kUChunk; ++cc) {
            const T* Uc = &U[min(c0 + cc, ncols - 1)][0];   // U is staged transposed: U[col][s]
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                T acc = x[q][cc];
#pragma unroll
                for (int s = 0; s < NB; ++s) acc = acc - l[q][s] * Uc[s];
                x[q][cc] = acc;
            }
        }
        const int nc = min(kUChunk, ncols - c0);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            if (!act[q]) continue;
            if (nc == kUChunk) {
#pragma unroll
                for (int cc = 0; cc < kUChunk; ++cc) A[rows[q] + (long long)(right0 + c0 + cc) * lda] = x[q][cc];
            } else {
                for (int cc = 0; cc < nc; ++cc) {
                    T v = x[q][0];
#pragma unroll
                    for (int k = 1; k < kUChunk; ++k) v = (cc == k) ? x[q][k] : v;
                    A[rows[q] + (long long)(right0 + c0 + cc) * lda] = v;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q)
#pragma unroll
            for (int cc = 0; cc < kUChunk; ++cc) x[q][cc] = y[q][cc];
    }
}

// Column loop of one block, as a shift register: at step j, reg[q][s] holds
// block column j+s of row row_of(q); finished columns go to memory (and to the
// LDS copy `fin`) at once, so every register index is a compile-time constant
// and the loop is not unrolled.
template <typename T, int NB, int RPT, int OCC>
__global__ __launch_bounds__(kPanelThreads) void panel_kernel(PanelArgs<T> a) {
    typedef Xch<T, NB> X;
    __shared__ PanelShared<T, NB, RPT> sh;
    const int tid = threadIdx.x;
    const int g = blockIdx.x;
    const int P = gridDim.x;
    const int R = kPanelThreads * RPT;
    const int m = a.m, w = a.w;
    const long long lda = a.lda;
    T* __restrict__ A = a.A;
    unsigned epoch = 0;            // full-barrier count

    if (g == 0 && tid == 0 && a.sync_next) {
        a.sync_next[0] = 0u;   // counter of the next launch's slot (its previous user has finished)
    }
    if (tid < NB) { sh.prow[NB + tid] = T(0); sh.drow[NB + tid] = T(0); }

    auto row_of = [&](int q) { return g * R + q * kPanelThreads + tid; };
    // finished column t (< NB) of the current block, own row q
    auto fin_get = [&](int t, int q, int cb) -> T {
        if constexpr (FinCfg<T, NB, RPT>::lds) return sh.fin[t][q * kPanelThreads + tid];
        else return A[min(row_of(q), m - 1) + (long long)(cb + t) * lda];
    };
    auto fin_set = [&](int t, int q, T v) {
        if constexpr (FinCfg<T, NB, RPT>::lds) sh.fin[t][q * kPanelThreads + tid] = v;
    };

    for (int cb = 0; cb < w; cb += NB) {
        const int nbw = (w - cb) < NB ? (w - cb) : NB;
        T reg[RPT][NB];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = row_of(q);
            const T* rp = A + min(i, m - 1);        // clamped: unconditional loads, select below
#pragma unroll
            for (int s = 0; s < NB; ++s) {
                const T v = rp[(long long)(cb + min(s, nbw - 1)) * lda];
                reg[q][s] = (i < m && s < nbw) ? v : T(0);
            }
        }

#pragma unroll 1
        for (int j = 0; j < nbw; ++j) {
            const int d = cb + j;
            const unsigned tag = a.tag_base + (unsigned)d;
            unsigned long long* xa = a.xch + (size_t)(d & 1) * X::PAR;     // this step's parity area
            // 1. local arg-max of |a| over rows >= d (current column = slot 0)
            T bv = T(-1);
            int bi = 0x7fffffff;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = row_of(q);
                if (i >= d && i < m) argmax_merge(bv, bi, dabs(reg[q][0]), i);
            }
            wave_argmax(bv, bi);
            if ((tid & (kWave - 1)) == 0) { sh.red_v[tid / kWave] = bv; sh.red_i[tid / kWave] = bi; }
            __syncthreads();
            if (tid == 0) {
#pragma unroll
                for (int wv = 1; wv < kPanelThreads / kWave; ++wv) argmax_merge(bv, bi, sh.red_v[wv], sh.red_i[wv]);
                sh.win_i = bi;
                unsigned long long* slot = xa + (size_t)g * X::SW;
                xstore(&slot[0], tagged(tag, (unsigned)bi));
                put_value(&slot[1], bv, tag);
            }
            __syncthreads();
            // 2. publish the local winner's block row and, from its owner, row d:
            //    finished columns < j from the LDS copy, the register part at
            //    positions j..j+NB-1 (slots hold 2*NB values)
            {
                const int wi = sh.win_i;
                if (wi == 0x7fffffff && tid < NB)      // no candidate here: a zero row completes the slot
                    put_value(&xa[(size_t)g * X::SW + 1 + X::WPV + tid * X::WPV], T(0), tag);
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int i = row_of(q);
                    if (i == wi || i == d) {
#pragma unroll
                        for (int slot = 0; slot < 2; ++slot) {
                            const bool mine = slot == 0 ? (i == wi) : (i == d);
                            if (!mine) continue;
                            unsigned long long* dst = slot == 0 ? xa + (size_t)g * X::SW + 1 + X::WPV
                                                                : xa + (size_t)kMaxPanelWgs * X::SW;
                            for (int t = 0; t < j; ++t) put_value(&dst[t * X::WPV], fin_get(t, q, cb), tag);
#pragma unroll
                            for (int s = 0; s < NB; ++s) put_value(&dst[(j + s) * X::WPV], reg[q][s], tag);
                        }
                    }
                }
            }
            // 3. gather every work-group's candidate and row d: poll the tagged
            //    words until all carry this step's tag (bounded wait)
            {
                const int nslot = P * X::SR;
                const int total = nslot + X::DR;
                constexpr int kMaxPer = (kMaxPanelWgs * X::SR + X::DR + kPanelThreads - 1) / kPanelThreads;
                unsigned done = 0u;                       // bit u: word tid + u*threads is in
                const long long t0 = wall_clock64();
                for (;;) {
                    int ok = 1;
#pragma unroll
                    for (int u = 0; u < kMaxPer; ++u) {
                        const int e2 = tid + u * kPanelThreads;
                        if (e2 < total && !(done & (1u << u))) {
                            const unsigned long long* src = (e2 < nslot)
                                ? xa + (size_t)(e2 / X::SR) * X::SW + (e2 % X::SR)
                                : xa + (size_t)kMaxPanelWgs * X::SW + (e2 - nslot);
                            const unsigned long long wv = xload(src);
                            if ((unsigned)(wv >> 32) == tag) { sh.xbuf[e2] = (unsigned)wv; done |= 1u << u; }
                            else ok = 0;
                        }
                    }
                    // bit 0: some word still stale; bit 1: time limit passed or another work-group failed
                    int st = ok ? 0 : 1;
                    if (tid == 0 && ((wall_clock64() - t0 > a.spin_limit) || xload(a.sync + 1) != 0u)) st |= 2;
                    st = __syncthreads_or(st);
                    if (!(st & 1)) break;
                    if (st & 2) {
                        if (tid == 0) xstore(a.sync + 1, 1u);
                        return;
                    }
                }
            }
            // 4. global winner (same decision in every work-group)
            if (tid < kWave) {
                T v = T(-1);
                int i = 0x7fffffff, gg = 0x7fffffff;
                for (int c = tid; c < P; c += kWave) {
                    const unsigned* sw = &sh.xbuf[c * X::SR];
                    const int ci = (int)sw[0];
                    const T cv = get_value(&sw[1], (T*)nullptr);
                    if (cv > v || (cv == v && ci < i)) { v = cv; i = ci; gg = c; }
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    T ov = __shfl_xor(v, off, kWave);
                    int oi = __shfl_xor(i, off, kWave);
                    int og = __shfl_xor(gg, off, kWave);
                    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; gg = og; }
                }
                if (tid == 0) {
                    if (i == 0x7fffffff) { i = d; gg = -1; }   // no finite candidate: keep row d
                    sh.win_i = i;
                    sh.win_g = gg;
                }
            }
            __syncthreads();
            const int p = sh.win_i;
            const int wg = sh.win_g;
            if (tid < NB) {
                sh.drow[tid] = get_value(&sh.xbuf[nslot_words<X>(P) + tid * X::WPV], (T*)nullptr);
                sh.prow[tid] = (wg >= 0) ? get_value(&sh.xbuf[wg * X::SR + 1 + X::WPV + tid * X::WPV], (T*)nullptr)
                                         : sh.drow[tid];
            }
            if (tid == 0) {
                sh.piv[d] = p;
                if (g == 0) {
                    a.ipiv[d] = a.row_base + p;
                    if (a.ipiv_rel) a.ipiv_rel[d] = p;
                }
            }
            __syncthreads();
            const T piv = sh.prow[j];
            if (piv == T(0) && g == 0 && tid == 0 && a.info) atomicCAS(a.info, 0, a.info_col_base + d + 1);
            // 5. rows d and p: the finished columns go to memory and to the LDS
            //    copy (columns >= j written too are rewritten when their own step
            //    stores them), the rest replaces the register block
            if (p != d) {
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int i = row_of(q);
                    if (i == p || i == d) {
                        const int so = (i == p) ? 0 : 2 * NB;       // sh.drow | sh.prow
                        const T* src = sh.drow + so;
#pragma unroll
                        for (int t = 0; t < NB; ++t) A[i + (long long)(cb + min(t, nbw - 1)) * lda] = src[min(t, nbw - 1)];
                        for (int t = 0; t < j; ++t) fin_set(t, q, src[t]);
#pragma unroll
                        for (int s = 0; s < NB; ++s) reg[q][s] = src[j + s];
                    }
                }
            }
            // 6. scale, rank-1 update, store column j, shift
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = row_of(q);
                if (i > d && i < m) {
                    T l = reg[q][0];
                    if (piv != T(0)) l = l / piv;
                    reg[q][0] = l;
#pragma unroll
                    for (int s = 1; s < NB; ++s) reg[q][s] = reg[q][s] - l * sh.prow[j + s];
                }
                if (i < m) A[i + (long long)d * lda] = reg[q][0];
                fin_set(j, q, reg[q][0]);
#pragma unroll
                for (int s = 0; s + 1 < NB; ++s) reg[q][s] = reg[q][s + 1];
                reg[q][NB - 1] = T(0);
            }
        }

        const bool more_cols = (w - cb - nbw) > 0 || cb > 0;
        if (more_cols) {
            const int gd = cb / R;     // owner of the block's diagonal rows
            if (g == gd) {
                __syncthreads();       // this work-group's stores of the block are visible to it
                for (int e = tid; e < NB * NB; e += kPanelThreads) {
                    const int r = e % NB, c = e / NB;
                    sh.L[r][c] = (r < nbw && c < nbw) ? A[(cb + r) + (long long)(cb + c) * lda] : T(0);
                }
                if (tid < kWave) compose_block_moves<NB>(sh.piv + cb, nbw, cb, sh.bmv, sh.slot_row, sh.content);
                __syncthreads();
                block_swap_trsm<T, NB>(A, lda, w, cb, nbw, sh.bmv, sh.L);
            }
            if (grid_barrier(a.sync, a.sync + 1, ++epoch, a.spin_limit)) return;
            // in-panel trailing update of my rows below the block: A[i, right] -= L[i, blk] U[blk, right]
            const int right0 = cb + nbw;
            const int ncols = w - right0;
            if (ncols > 0) {
                for (int e = tid; e < NB * ncols; e += kPanelThreads) {
                    const int s = e % NB, cc = e / NB;
                    sh.U[cc][s] = (s < nbw) ? A[(cb + s) + (long long)(right0 + cc) * lda] : T(0);
                }
                __syncthreads();
                int rows[RPT];
                bool any = false;
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int i = g * R + q * kPanelThreads + tid;
                    rows[q] = (i >= right0 && i < m) ? i : -1;
                    any |= rows[q] >= 0;
                }
                if (any) inpanel_update<T, NB, RPT>(A, lda, rows, cb, nbw, right0, ncols, sh.U, sh.fin);
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
    if (rpt == 1) hipLaunchKernelGGL((panel_kernel<T, NB, 1, 1>), dim3(wgs), block, 0, stream, args);
    else if (rpt == 2) hipLaunchKernelGGL((panel_kernel<T, NB, 2, 1>), dim3(wgs), block, 0, stream, args);
    else if (rpt <= 4) hipLaunchKernelGGL((panel_kernel<T, NB, 4, 1>), dim3(wgs), block, 0, stream, args);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int panel_max_rows_per_wg() { return kPanelThreads * 4; }
int panel_threads() { return kPanelThreads; }

template int launch_panel<double>(const PanelArgs<double>&, int, hipStream_t);
template int launch_panel<float>(const PanelArgs<float>&, int, hipStream_t);

}  // namespace lu
