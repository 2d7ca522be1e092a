// Solves with the packed LU factor (LAPACK getrs semantics: x = U^-1 L^-1 P b)
// and the FP64 side of iterative refinement.
//
// Triangular solves are "sync-free": the rows are cut into 64-row blocks, each
// with a ready flag, and work-groups are launched in block order (the LU
// solves take two consecutive blocks per work-group, the Cholesky solves one).
// A work-group accumulates L(r, c) x(c) for every finished block c before its
// own as soon as c's flag shows the current epoch, then solves its diagonal
// part in one wave and publishes its x values, then its flags.  A work-group
// only waits for lower-numbered blocks, which the hardware dispatched before
// it, so the grid always makes progress; every wait is bounded by a
// wall-clock limit that sets an error word instead of hanging.
#include "common.hpp"
#include "kernels.hpp"

namespace lu {

namespace {

constexpr int kRB = kTrsvRows;   // rows per triangular block
constexpr int kThreads = 256;    // 4 column groups x 64 rows

// Wait until a block's ready flag shows `epoch` (relaxed device-scope polls;
// the block's x values are read with device-coherent loads afterwards).
__device__ __forceinline__ bool wait_flag(const int* flag, int epoch, unsigned* err, long long limit) {
    __shared__ int s_fail;
    if (threadIdx.x == 0) {
        int fail = 0;
        const long long t0 = wall_clock64();
        unsigned spins = 0;
        // the error word and the clock every 16th poll: a poll is one round
        // trip to the coherence point, and a flag usually arrives within a few
        while (xload(flag) != epoch) {
            if ((++spins & 15u) != 0u) continue;
            if (xload(err) != 0u) { fail = 1; break; }
            if (wall_clock64() - t0 > limit) {
                xstore(err, 1u);
                fail = 1;
                break;
            }
        }
        s_fail = fail;
    }
    __syncthreads();
    return s_fail != 0;
}

// Publish x(r) and then its flag: the x stores complete before the flag store.
template <typename T>
__device__ __forceinline__ void publish(T* x, int row, T y, bool valid, int* flag, int epoch) {
    if (valid) xstore(&x[row], y);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) xstore(flag, epoch);
}

// LU solves: a work-group solves two consecutive blocks (128 rows), so the
// chain pays one publish / poll / fetch round trip per 128 rows instead of
// per 64.  Wave 0 polls, copies finished x values into LDS, holds both blocks'
// rows (lane i: rows i and 64 + i) for the 128-step substitution and
// publishes; 512 threads (4 column groups x 128 rows) prefetch the finished
// pairs' coefficients and accumulate.  A wave's loads complete in issue order,
// so a poll issued behind a prefetch waits for it: in FP32 wave 0 is a control
// wave of its own, with no prefetch.  In FP64 wave 0 also accumulates: a
// ninth wave would cap the registers at 168 per lane, and the FP64 kernel then
// spills (measured slower than the wait behind its own prefetch).
constexpr int kPR = 2 * kRB;               // rows per LU-solve work-group
template <typename T>
struct Pair {
    static constexpr bool own_ctl = sizeof(T) == 4;   // a control wave of its own
    static constexpr int acc = 512;                   // accumulating threads
    static constexpr int first = own_ctl ? kRB : 0;   // the first of them
    static constexpr int threads = first + acc;
    static constexpr int groups = acc / kPR;          // 4 (the partial sums of sum_parts)
    static constexpr int per = kPR / groups;          // columns per thread per finished pair
};

// Column loads of one wave: a column, uniform in the wave, as a buffer
// resource (scalar registers); element r of it is at byte offset
// r * sizeof(T), the one vector operand.  (Generic 64-bit addresses per load
// would cost two vector registers each, which the compiler keeps live across
// the wait loop.)  Resource: stride 0 (raw offsets), 2^31 - 1 bytes of range,
// and word 3 = 0x00020000, the 32-bit data format that gfx9 untyped buffer
// loads need (a zero format reads as zero).
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t cols_rsrc(const T* c0) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(c0), (short)0, 0x7fffffff, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T ld_rsrc(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}

// a(r, c) with the row and column clamped into the n x n matrix: every lane
// loads from a valid address, so no branch is wrapped around the load (a
// conditional load is compiled as a branch, and the loads of a prefetch then
// stop overlapping); callers discard or zero what lies outside
template <typename T>
__device__ __forceinline__ T ld_in(const T* a, long long lda, int r, int c, int n) {
    return a[min(r, n - 1) + (long long)min(c, n - 1) * lda];
}

template <typename T>
__device__ __forceinline__ T sum_parts(const T (&part)[4][kPR], int i) {
    return (part[0][i] + part[1][i]) + (part[2][i] + part[3][i]);
}

// kRB serial substitution steps of a wave: at step sc, the chain value c of
// lane sc (final by then) is broadcast and lanes on the unsolved side of sc
// (below it, or above it when Up) subtract coef(sc) * c_sc; with Side, every
// lane's second value (rows of the other block) subtracts side(sc) * c_sc.
// coef(sc) = a[sc * lds + off_c + lane], side(sc) = a[sc * lds + off_s + lane],
// in LDS.  The coefficients are fetched kCh steps ahead, and scheduling
// barriers keep the compiler from moving the fetch of the next kCh steps
// behind the current ones: each step then waits only for its multiply-add
// and broadcast, never for an LDS round trip.
template <typename T, bool Up, bool Side>
__device__ __forceinline__ void chain_steps(const T* a, int lds, int off_c, int off_s, T& c, T& side) {
    constexpr int kCh = 8, kNch = kRB / kCh;
    const int lane = threadIdx.x;
    T cc[kCh], cs[kCh];
    auto fetch = [&](int ch, T (&vc)[kCh], T (&vs)[kCh]) {
#pragma unroll
        for (int k = 0; k < kCh; ++k) {
            const int sc = Up ? kRB - 1 - (ch * kCh + k) : ch * kCh + k;
            vc[k] = a[sc * lds + off_c + lane];
            if constexpr (Side) vs[k] = a[sc * lds + off_s + lane];
        }
    };
    fetch(0, cc, cs);
#pragma unroll
    for (int ch = 0; ch < kNch; ++ch) {
        T nc[kCh], ns[kCh];
        if (ch + 1 < kNch) fetch(ch + 1, nc, ns);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < kCh; ++k) {
            const int sc = Up ? kRB - 1 - (ch * kCh + k) : ch * kCh + k;
            const T xs = lane_t(c, sc);                    // lane sc's value (sc is uniform)
            c = (Up ? lane < sc : lane > sc) ? c - cc[k] * xs : c;
            if constexpr (Side) side = side - cs[k] * xs;
        }
        __builtin_amdgcn_sched_barrier(0);
        if (ch + 1 < kNch) {
#pragma unroll
            for (int k = 0; k < kCh; ++k) {
                cc[k] = nc[k];
                if constexpr (Side) cs[k] = ns[k];
            }
        }
    }
}

// Wave 0 waits for pair p's flag (raised after both of its blocks' x values
// completed) and copies those values (nvalid of them) into LDS; the other waves
// meet it at the barrier.  Every wave of every waiting work-group used to load
// the values itself: one copy per work-group cuts the requests to the few
// cache lines that all of them want at the same moment.
template <typename T>
__device__ __forceinline__ bool wait_fetch_pair(const int* flag, int epoch, unsigned* err, long long limit,
                                                const T* xp, int nvalid, T* xl) {
    __shared__ int s_fail;
    const int lane = threadIdx.x;
    if (lane < kRB) {
        int fail = 0;
        const long long t0 = wall_clock64();
        unsigned spins = 0;
        // the flag, the error word and the clock are wave-uniform; as in
        // wait_flag, the error word and the clock every 16th poll
        while (xload(flag) != epoch) {
            if ((++spins & 15u) != 0u) continue;
            if (xload(err) != 0u) { fail = 1; break; }
            if (wall_clock64() - t0 > limit) {
                if (lane == 0) xstore(err, 1u);
                fail = 1;
                break;
            }
        }
        if (!fail) {
            xl[lane] = lane < nvalid ? xload(&xp[lane]) : T(0);
            xl[kRB + lane] = kRB + lane < nvalid ? xload(&xp[kRB + lane]) : T(0);
        }
        if (lane == 0) s_fail = fail;
    }
    __syncthreads();
    return s_fail != 0;
}

// Publish both blocks of a pair: x values, then (after they completed) the
// flags of block 2w and, if it exists, block 2w + 1.
template <typename T>
__device__ __forceinline__ void publish_pair(T* x, int n, int r0, T y0, T y1, int* flags, int w, int nblk,
                                             int epoch) {
    const int tid = threadIdx.x;
    if (tid < kRB) {
        if (r0 + tid < n) xstore(&x[r0 + tid], y0);
        if (r0 + kRB + tid < n) xstore(&x[r0 + kRB + tid], y1);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) xstore(&flags[2 * w], epoch);
    if (tid == 1 && 2 * w + 1 < nblk) xstore(&flags[2 * w + 1], epoch);
}

// L y = b for a pair of blocks.  Unit: L has a unit diagonal (the LU factor).
// Otherwise (a Cholesky factor) the pair's own part is solved as L' z = c with
// L' = L D^-1 (each column divided by its diagonal entry, unit diagonal) and
// then y = D^-1 z, which keeps the divisions off the serial chain.
template <typename T, bool Unit>
__device__ __forceinline__ void trsv_lower_pair(const T* __restrict__ LU, long long lda, int n, T* __restrict__ x,
                                                int* flags, int epoch, unsigned* err, long long limit) {
    constexpr int kPThreads = Pair<T>::threads, kPG = Pair<T>::groups, kPPerT = Pair<T>::per;
    __shared__ T part[kPG][kPR];
    __shared__ T La[kRB][kPR];     // La[s][i] = L(r0 + i, r0 + s) (/ L(r0 + s, r0 + s)): the first block's columns
    __shared__ T Lb[kRB][kRB];     // Lb[s][i] = L(r0 + 64 + i, r0 + 64 + s) (scaled alike): the second block's diagonal
    __shared__ T dg[kPR];          // L(r0 + k, r0 + k) (not Unit)
    const int w = blockIdx.x;
    const int nblk = (n + kRB - 1) / kRB;
    const int r0 = w * kPR;
    const int tid = threadIdx.x;
    const bool acc_t = tid >= Pair<T>::first;         // an accumulating thread: row i, column group g
    const int at = acc_t ? tid - Pair<T>::first : 0;
    const int i = at % kPR, g = at / kPR;
    const int row = r0 + i;
    // both blocks' right-hand sides, loaded before any wait (nothing else writes them)
    const T b0 = x[min(r0 + tid % kRB, n - 1)];     // used only by wave 0, for rows inside the matrix
    const T b1 = x[min(r0 + kRB + tid % kRB, n - 1)];
    // the diagonal part does not depend on other blocks: stage it first
    // (entries outside the matrix as zero; not Unit, scaled by the column's
    // diagonal entry, entries on or above the diagonal zero)
    if constexpr (!Unit) {
        if (tid < kPR) {
            const T v = ld_in(LU, lda, r0 + tid, r0 + tid, n);
            dg[tid] = (r0 + tid < n) ? v : T(0);
        }
        __syncthreads();
    }
    if (acc_t) {
        for (int sc = g; sc < kRB; sc += kPG) {
            const T v = ld_in(LU, lda, row, r0 + sc, n);
            if constexpr (Unit) La[sc][i] = (row < n && r0 + sc < n) ? v : T(0);
            else La[sc][i] = (row < n && i > sc) ? v / dg[sc] : T(0);
        }
    }
    for (int e = tid; e < kRB * kRB; e += kPThreads) {
        const int sc = e / kRB, ii = e % kRB;
        const int rr = r0 + kRB + ii, cc = r0 + kRB + sc;
        const T v = ld_in(LU, lda, rr, cc, n);
        if constexpr (Unit) Lb[sc][ii] = (rr < n && cc < n) ? v : T(0);
        else Lb[sc][ii] = (rr < n && ii > sc) ? v / dg[kRB + sc] : T(0);
    }
    // this thread's columns of the finished pair p (inside the matrix, since
    // p < w; rows past n load row n - 1 and their sums are discarded).  The
    // next pair's are loaded right after this pair's are used, so they are
    // in flight during the next wait.
    // (g is uniform in a wave, so each column address is scalar)
    const int gu = __builtin_amdgcn_readfirstlane(g);
    const int voff = min(row, n - 1) * (int)sizeof(T);
    auto load_l = [&](int p, T (&lv)[kPPerT]) {
#pragma unroll
        for (int u = 0; u < kPPerT; ++u)
            lv[u] = ld_rsrc<T>(cols_rsrc(LU + (long long)(p * kPR + gu + kPG * u) * lda), voff, 0);
    };
    __shared__ T xl[2][kPR];       // the x values of a finished pair (double-buffered)
    T acc = T(0);
    T lv[kPPerT];
    if (w > 0 && acc_t) load_l(0, lv);
    for (int p = 0; p < w; ++p) {
        T* xv = xl[p & 1];
        if (wait_fetch_pair(&flags[2 * p], epoch, err, limit, x + p * kPR, kPR, xv)) return;
        if (acc_t) {
#pragma unroll
            for (int u = 0; u < kPPerT; ++u) acc += lv[u] * xv[g + kPG * u];
            if (p + 1 < w) load_l(p + 1, lv);
        }
    }
    if (acc_t) part[g][i] = acc;
    __syncthreads();
    T y0 = T(0), y1 = T(0);
    if (tid < kRB) {
        y0 = (r0 + tid < n) ? b0 - sum_parts(part, tid) : T(0);
        y1 = (r0 + kRB + tid < n) ? b1 - sum_parts(part, kRB + tid) : T(0);
        // rows and columns outside the matrix hold zero and change nothing
        T none = T(0);
        chain_steps<T, false, true>(&La[0][0], kPR, 0, kRB, y0, y1);    // the first block's columns
        chain_steps<T, false, false>(&Lb[0][0], kRB, 0, 0, y1, none);   // the second block's diagonal
        if constexpr (!Unit) {
            y0 = (r0 + tid < n) ? y0 / dg[tid] : T(0);
            y1 = (r0 + kRB + tid < n) ? y1 / dg[kRB + tid] : T(0);
        }
    }
    publish_pair(x, n, r0, y0, y1, flags, w, nblk, epoch);
}

template <typename T>
__global__ __launch_bounds__(Pair<T>::threads) void trsv_lower_unit_kernel(const T* __restrict__ LU, long long lda, int n,
                                                                     T* __restrict__ x, int* flags, int epoch,
                                                                     unsigned* err, long long limit) {
    trsv_lower_pair<T, true>(LU, lda, n, x, flags, epoch, err, limit);
}

// Cholesky: L y = b with the non-unit lower factor
template <typename T>
__global__ __launch_bounds__(Pair<T>::threads) void trsv_chol_lower_kernel(const T* __restrict__ L, long long lda, int n,
                                                                     T* __restrict__ x, int* flags, int epoch,
                                                                     unsigned* err, long long limit) {
    trsv_lower_pair<T, false>(L, lda, n, x, flags, epoch, err, limit);
}

template <typename T>
__global__ __launch_bounds__(Pair<T>::threads) void trsv_upper_kernel(const T* __restrict__ LU, long long lda, int n,
                                                                T* __restrict__ x, int* flags, int epoch,
                                                                unsigned* err, long long limit) {
    constexpr int kPThreads = Pair<T>::threads, kPG = Pair<T>::groups, kPPerT = Pair<T>::per;
    // The pair's own part is solved as U' z = c with U' = U D^-1 (each column
    // divided by its diagonal entry, so U' has a unit diagonal) and then
    // x = D^-1 z: the divisions leave the serial chain, which is left with
    // one multiply-add per step.  Scaled entries strictly above the diagonal:
    __shared__ T part[kPG][kPR];
    __shared__ T Uc[kRB][kPR];     // Uc[s][i] = U(r0 + i, r0 + 64 + s) / U(r0 + 64 + s, r0 + 64 + s), all 128 rows
    __shared__ T Ut[kRB][kRB];     // Ut[s][i] = U(r0 + i, r0 + s) / U(r0 + s, r0 + s), the first block
    __shared__ T dg[kPR];          // U(r0 + k, r0 + k)
    const int nblk = (n + kRB - 1) / kRB;
    const int npair = (nblk + 1) / 2;
    const int w = npair - 1 - (int)blockIdx.x;       // bottom pair first
    const int r0 = w * kPR;
    const int tid = threadIdx.x;
    const bool acc_t = tid >= Pair<T>::first;         // an accumulating thread: row i, column group g
    const int at = acc_t ? tid - Pair<T>::first : 0;
    const int i = at % kPR, g = at / kPR;
    const int row = r0 + i;
    const T b0 = x[min(r0 + tid % kRB, n - 1)];     // used only by wave 0, for rows inside the matrix
    const T b1 = x[min(r0 + kRB + tid % kRB, n - 1)];
    if (tid < kPR) {
        const T v = ld_in(LU, lda, r0 + tid, r0 + tid, n);
        dg[tid] = (r0 + tid < n) ? v : T(0);
    }
    __syncthreads();
    // entries on or below the diagonal and outside the matrix are zero (the
    // quotients of those are discarded)
    if (acc_t) {
        for (int sc = g; sc < kRB; sc += kPG) {
            const int cc = r0 + kRB + sc;
            const T v = ld_in(LU, lda, row, cc, n) / dg[kRB + sc];
            Uc[sc][i] = (cc < n && i < kRB + sc) ? v : T(0);
        }
    }
    for (int e = tid; e < kRB * kRB; e += kPThreads) {
        const int sc = e / kRB, ii = e % kRB;
        const int cc = r0 + sc;
        const T v = ld_in(LU, lda, r0 + ii, cc, n) / dg[sc];
        Ut[sc][ii] = (cc < n && ii < sc) ? v : T(0);
    }
    // pair p > w, loaded right after pair p + 1 is used (as in the lower
    // solve); rows past n are discarded, and columns past n (only in the
    // bottom pair) are zeroed when used, with their x
    // (scalar column addresses, as in the lower solve)
    const int gu = __builtin_amdgcn_readfirstlane(g);
    const int voff = min(row, n - 1) * (int)sizeof(T);
    auto load_u = [&](int p, T (&lv)[kPPerT]) {
#pragma unroll
        for (int u = 0; u < kPPerT; ++u)
            lv[u] = ld_rsrc<T>(cols_rsrc(LU + (long long)min(p * kPR + gu + kPG * u, n - 1) * lda), voff, 0);
    };
    __shared__ T xl[2][kPR];       // the x values of a finished pair (double-buffered)
    T acc = T(0);
    T lv[kPPerT];
    if (w < npair - 1 && acc_t) load_u(npair - 1, lv);
    for (int p = npair - 1; p > w; --p) {
        T* xv = xl[p & 1];
        // values past n read as zero
        if (wait_fetch_pair(&flags[2 * p], epoch, err, limit, x + p * kPR, min(kPR, n - p * kPR), xv)) return;
        if (acc_t) {
#pragma unroll
            for (int u = 0; u < kPPerT; ++u) {
                const T l = p * kPR + g + kPG * u < n ? lv[u] : T(0);
                acc += l * xv[g + kPG * u];
            }
            if (p - 1 > w) load_u(p - 1, lv);
        }
    }
    if (acc_t) part[g][i] = acc;
    __syncthreads();
    T y0 = T(0), y1 = T(0);
    if (tid < kRB) {
        const bool in0 = r0 + tid < n, in1 = r0 + kRB + tid < n;
        y0 = in0 ? b0 - sum_parts(part, tid) : T(0);
        y1 = in1 ? b1 - sum_parts(part, kRB + tid) : T(0);
        // unit upper substitution on the scaled entries, bottom up; a column
        // outside the matrix has z = 0 and zero entries
        T none = T(0);
        chain_steps<T, true, true>(&Uc[0][0], kPR, kRB, 0, y1, y0);     // the second block's columns
        chain_steps<T, true, false>(&Ut[0][0], kRB, 0, 0, y0, none);    // the first block's diagonal
        y0 = in0 ? y0 / dg[tid] : T(0);
        y1 = in1 ? y1 / dg[kRB + tid] : T(0);
    }
    publish_pair(x, n, r0, y0, y1, flags, w, nblk, epoch);
}

// L^T x = y, bottom block first.  Element (i, j) of L^T is L[j + i*lda]: the
// off-diagonal blocks are read along j (contiguous) into LDS, transposed.
template <typename T>
__global__ __launch_bounds__(kThreads) void trsv_chol_upper_kernel(const T* __restrict__ L, long long lda, int n,
                                                                    T* __restrict__ x, int* flags, int epoch,
                                                                    unsigned* err, long long limit) {
    __shared__ T part[4][kRB];
    // this block's diagonal part, solved as U' z = c with U' = U D^-1 (unit
    // diagonal), U = L^T, then x = D^-1 z (the divisions off the serial chain)
    __shared__ T Ud[kRB][kRB + 1];       // Ud[s][i] = L^T(i, s) / L(s, s) = L(s, i) / L(s, s), i < s
    __shared__ T dg[kRB];                // L(r0 + i, r0 + i)
    __shared__ T S[kRB][kRB + 1];        // S[i][jj] = L^T(i, j0 + jj) of the block being applied
    const int nblk = (n + kRB - 1) / kRB;
    const int r = nblk - 1 - (int)blockIdx.x;
    const int tid = threadIdx.x, i = tid % kRB, g = tid / kRB;
    const int r0 = r * kRB;
    const int row = r0 + i;
    const int nb = min(kRB, n - r0);
    // this block's right-hand side, loaded before any wait (nothing else writes
    // it); loads below are unconditional from clamped addresses (a conditional
    // load compiles to a branch that waits for each round trip)
    const T b_row = x[min(row, n - 1)];            // used only for rows inside the matrix
    if (tid < kRB) {
        const T v = ld_in(L, lda, row, row, n);
        dg[i] = row < n ? v : T(0);
    }
    __syncthreads();
    // coalesced along the rows of L: thread (jj = tid % 64) reads L(r0 + jj, r0 + ii)
    for (int ii = g; ii < kRB; ii += 4) {
        const T v = ld_in(L, lda, r0 + i, r0 + ii, n);
        Ud[i][ii] = (i < nb && ii < i) ? v / dg[i] : T(0);
    }
    constexpr int kPerT = kRB / 4;
    // v[u] = L(j0 + i, r0 + g + 4u): row j0+i of L; entries outside the
    // matrix are never used (their x or their row is out of range)
    auto load_s = [&](int cb, T (&v)[kPerT]) {
        const int j0 = cb * kRB;
#pragma unroll
        for (int u = 0; u < kPerT; ++u) v[u] = ld_in(L, lda, j0 + i, r0 + g + 4 * u, n);
    };
    T acc = T(0);
    T sv[kPerT];
    if (r < nblk - 1) load_s(nblk - 1, sv);
    for (int cb = nblk - 1; cb > r; --cb) {
        T sn[kPerT];
        if (cb - 1 > r) load_s(cb - 1, sn);
        if (wait_flag(&flags[cb], epoch, err, limit)) return;
#pragma unroll
        for (int u = 0; u < kPerT; ++u) S[g + 4 * u][i] = sv[u];   // S[ii][jj]: row ii of L^T's block
        __syncthreads();
        if (row < n) {
            const int j0 = cb * kRB;
            const int nj = min(kRB, n - j0);
#pragma unroll
            for (int u = 0; u < kPerT; ++u)
                if (g + 4 * u < nj) acc += S[i][g + 4 * u] * xload(&x[j0 + g + 4 * u]);
        }
        __syncthreads();
        if (cb - 1 > r) {
#pragma unroll
            for (int u = 0; u < kPerT; ++u) sv[u] = sn[u];
        }
    }
    part[g][i] = acc;
    __syncthreads();
    T y = T(0);
    if (tid < kRB) {
        y = (row < n) ? b_row - ((part[0][i] + part[1][i]) + (part[2][i] + part[3][i])) : T(0);
        // rows and columns past a ragged block's end hold zero and change nothing
        T none = T(0);
        chain_steps<T, true, false>(&Ud[0][0], kRB + 1, 0, 0, y, none);
        y = (row < n) ? y / dg[i] : T(0);
    }
    publish(x, row, y, tid < kRB && row < n, &flags[r], epoch);
}

// P x for each right-hand side: chunk c's interchanges, chunks in order.
template <typename T>
__global__ __launch_bounds__(kThreads) void apply_chunk_moves_kernel(T* X, long long ldx, int n, int W,
                                                                      const int* moves) {
    T* x = X + (long long)blockIdx.x * ldx;
    const int nchunk = (n + W - 1) / W;
    const int tid = threadIdx.x;
    constexpr int kPer = (2 * kMovesMaxW + kThreads - 1) / kThreads;
    for (int c = 0; c < nchunk; ++c) {
        const int* mv = moves + (size_t)c * kMovesLen;
        const int base = c * W;
        const int ntop = mv[0], nex = mv[1];
        T v[kPer];
        int dst[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int s = tid + u * kThreads;
            dst[u] = -1;
            if (s < ntop) { dst[u] = mv[2 + 2 * s]; v[u] = x[base + mv[3 + 2 * s]]; }
            else if (s < ntop + nex) {
                const int e = s - ntop;
                dst[u] = mv[kMovesExtra + 2 * e];
                v[u] = x[base + mv[kMovesExtra + 1 + 2 * e]];
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            if (dst[u] >= 0) x[base + dst[u]] = v[u];
        __syncthreads();
    }
}

// partial[s][i] = sum over columns of slice s of A[i,j] * x[j]   (x == nullptr: |A[i,j]|)
__global__ __launch_bounds__(256) void gemv_partial_kernel(const double* __restrict__ A, long long lda, int n,
                                                           const double* __restrict__ x, double* partial,
                                                           int splits) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    const int per = (n + splits - 1) / splits;
    const int j0 = s * per, j1 = min(n, j0 + per);
    double acc = 0.0;
    if (i < n) {
        if (x) {
#pragma unroll 8
            for (int j = j0; j < j1; ++j) acc += A[i + (long long)j * lda] * x[j];
        } else {
#pragma unroll 8
            for (int j = j0; j < j1; ++j) acc += fabs(A[i + (long long)j * lda]);
        }
        partial[(long long)s * n + i] = acc;
    }
}

// The refinement's working copy and ||A||_inf in one pass over A:
// dst = (float)A, partial[s][i] = sum over the columns of slice s of |A[i,j]|.
__global__ __launch_bounds__(256) void convert_abs_partial_kernel(const double* __restrict__ A, long long lda, int n,
                                                                  float* __restrict__ dst, long long ldd,
                                                                  double* partial, int splits) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    const int per = (n + splits - 1) / splits;
    const int j0 = s * per, j1 = min(n, j0 + per);
    double acc = 0.0;
    if (i < n) {
#pragma unroll 8
        for (int j = j0; j < j1; ++j) {
            const double a = A[i + (long long)j * lda];
            dst[i + (long long)j * ldd] = (float)a;
            acc += fabs(a);
        }
        partial[(long long)s * n + i] = acc;
    }
}

__device__ __forceinline__ void atomic_max_abs(unsigned long long* out, double v) {
    // non-negative doubles order like their bit patterns; NaN bits sort above +inf
    atomicMax(out, (unsigned long long)__double_as_longlong(fabs(v)));
}

__global__ __launch_bounds__(256) void residual_finish_kernel(const double* partial, int splits, int n,
                                                              const double* b, double* r) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        double s = 0.0;
        for (int p = 0; p < splits; ++p) s += partial[(long long)p * n + i];
        r[i] = b[i] - s;
    }
}

__global__ __launch_bounds__(256) void rowsum_max_kernel(const double* partial, int splits, int n,
                                                         unsigned long long* out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        double s = 0.0;
        for (int p = 0; p < splits; ++p) s += partial[(long long)p * n + i];
        atomic_max_abs(out, s);
    }
}

__global__ __launch_bounds__(256) void amax_kernel(const double* x, int n, unsigned long long* out) {
    __shared__ double red[256];
    double m = 0.0;
    bool bad = false;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double a = fabs(x[i]);
        if (!(a <= 1.7976931348623157e308)) bad = true;
        m = fmax(m, a);
    }
    red[threadIdx.x] = bad ? __longlong_as_double(0x7ff8000000000000LL) : m;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long best = 0ull;
        for (int t = 0; t < 256; ++t) {
            const unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(red[t]));
            best = bits > best ? bits : best;
        }
        atomicMax(out, best);
    }
}

__global__ __launch_bounds__(256) void convert_kernel(const double* src, long long lds, float* dst, long long ldd,
                                                      int rows, int cols) {
    const long long total = (long long)rows * cols;
    for (long long e = blockIdx.x * 256ll + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
        const int i = (int)(e % rows);
        const long long j = e / rows;
        dst[i + j * ldd] = (float)src[i + j * lds];
    }
}

__global__ __launch_bounds__(256) void copy_kernel(const double* src, long long lds, double* dst, long long ldd,
                                                   int rows, int cols) {
    const long long total = (long long)rows * cols;
    for (long long e = blockIdx.x * 256ll + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
        const int i = (int)(e % rows);
        const long long j = e / rows;
        dst[i + j * ldd] = src[i + j * lds];
    }
}

__global__ __launch_bounds__(256) void axpy_kernel(double* x, const float* d, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = x[i] + (double)d[i];
}

__global__ __launch_bounds__(256) void fill_zero_kernel(unsigned* p, size_t words) {
    for (size_t e = blockIdx.x * 256ull + threadIdx.x; e < words; e += (size_t)gridDim.x * 256) p[e] = 0u;
}

inline int grid_for(long long work) {
    long long g = (work + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

int trsv_block_rows() { return kRB; }

template <typename T>
int launch_apply_chunk_moves(T* X, long long ldx, int n, int nrhs, int W, const int* moves, hipStream_t stream) {
    if (n <= 0 || nrhs <= 0) return 0;
    hipLaunchKernelGGL((apply_chunk_moves_kernel<T>), dim3(nrhs), dim3(kThreads), 0, stream, X, ldx, n, W, moves);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_trsv_lower_unit(const T* LU, long long lda, int n, T* x, int* flags, int epoch, unsigned* err,
                           long long spin_limit, hipStream_t stream) {
    if (n <= 0) return 0;
    const int npair = ((n + kRB - 1) / kRB + 1) / 2;
    hipLaunchKernelGGL((trsv_lower_unit_kernel<T>), dim3(npair), dim3(Pair<T>::threads), 0, stream, LU, lda, n, x, flags,
                       epoch, err, spin_limit);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_trsv_chol(const T* L, long long lda, int n, T* x, int* flags, int epoch_lower, int epoch_upper,
                     unsigned* err, long long spin_limit, hipStream_t stream) {
    if (n <= 0) return 0;
    const int nblk = (n + kRB - 1) / kRB;
    const int npair = (nblk + 1) / 2;
    hipLaunchKernelGGL((trsv_chol_lower_kernel<T>), dim3(npair), dim3(Pair<T>::threads), 0, stream, L, lda, n, x,
                       flags, epoch_lower, err, spin_limit);
    hipLaunchKernelGGL((trsv_chol_upper_kernel<T>), dim3(nblk), dim3(kThreads), 0, stream, L, lda, n, x, flags,
                       epoch_upper, err, spin_limit);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_trsv_upper(const T* LU, long long lda, int n, T* x, int* flags, int epoch, unsigned* err,
                      long long spin_limit, hipStream_t stream) {
    if (n <= 0) return 0;
    const int npair = ((n + kRB - 1) / kRB + 1) / 2;
    hipLaunchKernelGGL((trsv_upper_kernel<T>), dim3(npair), dim3(Pair<T>::threads), 0, stream, LU, lda, n, x, flags, epoch,
                       err, spin_limit);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_residual(const double* A, long long lda, int n, const double* x, const double* b, double* r,
                    double* partial, int splits, hipStream_t stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(gemv_partial_kernel, dim3((n + 255) / 256, splits), dim3(256), 0, stream, A, lda, n, x,
                       partial, splits);
    hipLaunchKernelGGL(residual_finish_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, partial, splits, n, b,
                       r);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_row_abs_sums(const double* A, long long lda, int n, double* partial, int splits, double* out_max,
                        hipStream_t stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(gemv_partial_kernel, dim3((n + 255) / 256, splits), dim3(256), 0, stream, A, lda, n,
                       (const double*)nullptr, partial, splits);
    hipLaunchKernelGGL(rowsum_max_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, partial, splits, n,
                       reinterpret_cast<unsigned long long*>(out_max));
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_convert_row_abs_sums(const double* A, long long lda, int n, float* dst, long long ldd, double* partial,
                                int splits, double* out_max, hipStream_t stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(convert_abs_partial_kernel, dim3((n + 255) / 256, splits), dim3(256), 0, stream, A, lda, n,
                       dst, ldd, partial, splits);
    hipLaunchKernelGGL(rowsum_max_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, partial, splits, n,
                       reinterpret_cast<unsigned long long*>(out_max));
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_amax(const double* x, int n, unsigned long long* out_bits, hipStream_t stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(amax_kernel, dim3(min(1024, (n + 255) / 256)), dim3(256), 0, stream, x, n, out_bits);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_convert_f64_f32(const double* src, long long lds, float* dst, long long ldd, int rows, int cols,
                           hipStream_t stream) {
    hipLaunchKernelGGL(convert_kernel, dim3(grid_for((long long)rows * cols)), dim3(256), 0, stream, src, lds, dst,
                       ldd, rows, cols);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_copy_f64(const double* src, long long lds, double* dst, long long ldd, int rows, int cols,
                    hipStream_t stream) {
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for((long long)rows * cols)), dim3(256), 0, stream, src, lds, dst, ldd,
                       rows, cols);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_axpy_f32_to_f64(double* x, const float* d, int n, hipStream_t stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(axpy_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, x, d, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_fill_zero(void* p, size_t bytes, hipStream_t stream) {
    const size_t words = bytes / 4;
    if (words == 0) return 0;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for((long long)words)), dim3(256), 0, stream,
                       reinterpret_cast<unsigned*>(p), words);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_apply_chunk_moves<double>(double*, long long, int, int, int, const int*, hipStream_t);
template int launch_apply_chunk_moves<float>(float*, long long, int, int, int, const int*, hipStream_t);
template int launch_trsv_lower_unit<double>(const double*, long long, int, double*, int*, int, unsigned*, long long,
                                            hipStream_t);
template int launch_trsv_lower_unit<float>(const float*, long long, int, float*, int*, int, unsigned*, long long,
                                           hipStream_t);
template int launch_trsv_chol<double>(const double*, long long, int, double*, int*, int, int, unsigned*, long long,
                                      hipStream_t);
template int launch_trsv_upper<double>(const double*, long long, int, double*, int*, int, unsigned*, long long,
                                       hipStream_t);
template int launch_trsv_upper<float>(const float*, long long, int, float*, int*, int, unsigned*, long long,
                                      hipStream_t);

}  // namespace lu
