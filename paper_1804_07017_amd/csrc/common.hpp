// Device helpers shared by the gfx950 kernels of the LU library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace lu {

constexpr int kWave = 64;

template <typename T> __device__ __forceinline__ T dabs(T x) { return x < T(0) ? -x : x; }
template <> __device__ __forceinline__ double dabs<double>(double x) { return fabs(x); }
template <> __device__ __forceinline__ float dabs<float>(float x) { return fabsf(x); }

// (value, index) arg-max with the smallest index winning ties; NaN never wins.
template <typename T>
__device__ __forceinline__ void argmax_merge(T& v, int& i, T ov, int oi) {
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
}

// Cross-lane moves by DPP (no LDS traffic): CTRL is a gfx9 dpp_ctrl code.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int x) { return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false); }
template <int CTRL>
__device__ __forceinline__ float dpp_t(float x) { return __int_as_float(dpp_i32<CTRL>(__float_as_int(x))); }
template <int CTRL>
__device__ __forceinline__ double dpp_t(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_i32<CTRL>((int)b), hi = dpp_i32<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ int lane_i32(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ float lane_t(float x, int l) { return __int_as_float(lane_i32(__float_as_int(x), l)); }
__device__ __forceinline__ double lane_t(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = lane_i32((int)b, l), hi = lane_i32((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <typename T, int CTRL>
__device__ __forceinline__ void dpp_argmax_step(T& v, int& i) {
    const T ov = dpp_t<CTRL>(v);
    const int oi = dpp_i32<CTRL>(i);
    argmax_merge(v, i, ov, oi);
}

// Arg-max over the 64 lanes of a wave (largest v, then smallest i), the
// result in every lane.  Butterflies inside 16-lane rows by DPP (quad
// permutations, then half-row and row mirrors), then the four row results are
// read as scalars and merged.  Every lane of the wave must be active.
template <typename T>
__device__ __forceinline__ void wave_argmax_all(T& v, int& i) {
    dpp_argmax_step<T, 0xB1>(v, i);     // quad_perm [1,0,3,2]
    dpp_argmax_step<T, 0x4E>(v, i);     // quad_perm [2,3,0,1]
    dpp_argmax_step<T, 0x141>(v, i);    // row_half_mirror
    dpp_argmax_step<T, 0x140>(v, i);    // row_mirror
    T rv = lane_t(v, 0);
    int ri = lane_i32(i, 0);
#pragma unroll
    for (int r = 1; r < 4; ++r) argmax_merge(rv, ri, lane_t(v, 16 * r), lane_i32(i, 16 * r));
    v = rv;
    i = ri;
}

template <typename T>
__device__ __forceinline__ void wave_argmax(T& v, int& i) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        T ov = __shfl_xor(v, off, kWave);
        int oi = __shfl_xor(i, off, kWave);
        argmax_merge(v, i, ov, oi);
    }
}

// Work-group barrier that orders LDS accesses only.  Unlike __syncthreads()
// it does not wait for this thread's outstanding global stores (the panel's
// exchange words carry their own tags, so nothing read across this barrier
// depends on them).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// OR of v over the work-group of `waves` wavefronts through LDS slots
// slots[2][waves]; callers alternate `parity` between consecutive calls so a
// slot is never rewritten before every wave has read it.
__device__ __forceinline__ int wg_or(int v, int* slots, int parity, int waves) {
    const int wave = threadIdx.x / 64;
    const int any = __any(v & 1) | (__any(v & 2) << 1) | (__any(v & 4) << 2);
    if ((threadIdx.x & 63) == 0) slots[parity * waves + wave] = any;
    lds_barrier();
    int r = 0;
    for (int w = 0; w < waves; ++w) r |= slots[parity * waves + w];
    return r;
}

// Device-coherent exchange words.  Agent-scope relaxed atomic loads and stores
// go to the device coherence point and bypass the non-coherent per-CU / per-XCD
// caches, so data published this way needs no cache write-back or invalidate.
template <typename T>
__device__ __forceinline__ void xstore(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T xload(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Scoped, fence-free forms used by the panel kernel.  Every access to data
// that another work-group of the launch reads or writes is a relaxed atomic
// at scope S; the panel uses S = __HIP_MEMORY_SCOPE_AGENT, the device
// coherence point (the per-CU L1 and the per-XCD L2 are bypassed).  Ordering
// then needs no cache write-back or invalidate (which, at agent scope, act on
// a whole XCD's L2 and stall the work beside the panel): a writer waits for
// its own accesses to complete (s_waitcnt) before it signals, and a reader
// issues its loads after it has seen the signal.
template <int S>
__device__ __forceinline__ void xstore_s(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ void xstore_s(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, S);
}
template <int S, typename U>
__device__ __forceinline__ U xload_s(const U* p) {
    return __hip_atomic_load(const_cast<U*>(p), __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ double cload(const double* p) {
    return __longlong_as_double((long long)xload_s<S>(reinterpret_cast<const unsigned long long*>(p)));
}
template <int S>
__device__ __forceinline__ float cload(const float* p) {
    return __uint_as_float(xload_s<S>(reinterpret_cast<const unsigned*>(p)));
}
template <int S>
__device__ __forceinline__ void cstore(double* p, double v) {
    xstore_s<S>(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}
template <int S>
__device__ __forceinline__ void cstore(float* p, float v) {
    xstore_s<S>(reinterpret_cast<unsigned*>(p), __float_as_uint(v));
}
// This wave's memory accesses have completed (at their scope's coherence
// point for the scoped atomics above).  The signal fences keep the compiler
// from moving memory operations across the wait.
__device__ __forceinline__ void wave_mem_drain() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Barrier among the nwg participating work-groups of one launch, without
// fences: every wave drains its accesses, then one arrival per work-group on
// a relaxed counter.  The counter and the error word are shared with launches
// of either scope, so they are always accessed at the device coherence point
// (a word must not be updated at one XCD's L2 by one launch and at the
// device coherence point by another).  The wait is bounded as in grid_barrier.
__device__ __forceinline__ bool grid_barrier_nofence(unsigned* counter, unsigned* err, unsigned epoch,
                                                     long long limit, int nwg) {
    constexpr int A = __HIP_MEMORY_SCOPE_AGENT;
    __shared__ int s_fail;
    wave_mem_drain();
    __syncthreads();
    if (threadIdx.x == 0 && nwg > 1) {
        const unsigned target = epoch * (unsigned)nwg;
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, A);
        int fail = 0;
        const long long t0 = wall_clock64();
        while (xload_s<A>(counter) < target) {
            if (xload_s<A>(err) != 0u) { fail = 1; break; }
            if (wall_clock64() - t0 > limit) {
                xstore_s<A>(err, 1u);
                fail = 1;
                break;
            }
        }
        s_fail = fail;
    } else if (threadIdx.x == 0) {
        s_fail = 0;
    }
    __syncthreads();
    return s_fail != 0;
}

// XCD (accelerator complex die) the calling wave runs on: hardware register
// XCC_ID, bits [3:0].
__device__ __forceinline__ int xcd_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15; }

// Device-wide barrier among the gridDim.x work-groups of one launch.  All of
// them must be resident at once (the host sizes the grid for that).  The
// counter starts at 0 for the launch; barrier number `epoch` (1-based) waits
// until the counter reaches epoch*gridDim.x.  The wait is bounded: past
// `limit` ticks of the constant-rate wall clock, or when another work-group
// has already failed, the error word is set and true is returned so that the
// caller exits instead of hanging.
//
// full = true : every wave makes its ordinary global writes visible
//               device-wide before arriving and re-reads device-wide data
//               after leaving (release / acquire fences at agent scope).
// full = false: only data exchanged through xstore/xload is ordered: each
//               wave waits for its own outstanding memory operations to
//               complete before the work-group arrives, and the counter is a
//               relaxed device-scope atomic.  No cache maintenance.
__device__ __forceinline__ bool grid_barrier(unsigned* counter, unsigned* err, unsigned epoch,
                                             long long limit, bool full = true) {
    __shared__ int s_fail;
    if (full) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    else __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0 && gridDim.x > 1) {   // a single work-group needs only its own barrier
        const unsigned target = epoch * gridDim.x;
        if (full) __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        else __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int fail = 0;
        const long long t0 = wall_clock64();
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) { fail = 1; break; }
            if (wall_clock64() - t0 > limit) {
                __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                fail = 1;
                break;
            }
        }
        s_fail = fail;
    } else if (threadIdx.x == 0) {
        s_fail = 0;
    }
    __syncthreads();
    if (full) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return s_fail != 0;
}

// Composition of a run of row interchanges into one gather/scatter.
//
// Steps t = 0..w-1 interchange rows t and p[t] (p[t] >= t, rows relative to
// the first row of the run).  Rows 0..w-1 are the "top" rows; rows >= w that
// some p[t] names are "extra" rows.  With
//   L(t)    = the latest step t' != t with p[t'] == t      (none: -1)
//   f(t)    = f(L(t)) if L(t) >= 0 else t   (the row whose data sits in top
//             row t when step t begins)
//   prev(t) = the latest step t' < t with p[t'] == p[t]    (none: -1)
// the result of all w interchanges is
//   top row t   <- f(t)                     if p[t] == t
//               <- f(prev(t)) or p[t]       otherwise (prev(t) >= 0 / < 0)
//   extra row e <- f(t) for the last step t with p[t] == e.
// One work-group computes this in LDS: L by atomic max, f by pointer
// jumping, prev by a bitonic sort of (p[t], t).  w <= kMovesMaxW.
//
// Output layout (int[kMovesLen]), rows relative to the run, only rows whose
// content changes:
//   [0] number of top moves, [1] number of extra moves,
//   [2 + 2s], [3 + 2s]                      (dst, src) of top move s
//   [kMovesExtra + 2e], [kMovesExtra+1+2e]  (dst, src) of extra move e

struct MovesScratch {
    int key[kMovesMaxW];       // sorted (p << 10 | t)
    int last_top[kMovesMaxW];
    int ptr_a[kMovesMaxW];
    int ptr_b[kMovesMaxW];
    int count_top, count_extra;
};

__device__ inline void compose_moves(const int* p, int w, int* moves, MovesScratch& s) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int t = tid; t < kMovesMaxW; t += nt) {
        s.last_top[t] = -1;
        s.key[t] = t < w ? ((p[t] << 10) | t) : 0x7fffffff;
    }
    if (tid == 0) { s.count_top = 0; s.count_extra = 0; }
    __syncthreads();
    for (int t = tid; t < w; t += nt) {
        int q = p[t];
        if (q < w && q != t) atomicMax(&s.last_top[q], t);
    }
    // bitonic sort of key[0..kMovesMaxW)
    for (int size = 2; size <= kMovesMaxW; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int i = tid; i < kMovesMaxW / 2; i += nt) {
                int lo = 2 * i - (i & (stride - 1));
                int hi = lo + stride;
                bool up = ((lo & size) == 0);
                int a = s.key[lo], b = s.key[hi];
                if ((a > b) == up) { s.key[lo] = b; s.key[hi] = a; }
            }
        }
    }
    __syncthreads();
    for (int t = tid; t < w; t += nt) s.ptr_a[t] = s.last_top[t] >= 0 ? s.last_top[t] : t;
    __syncthreads();
    int* cur = s.ptr_a;
    int* nxt = s.ptr_b;
    for (int round = 0; (1 << round) < w; ++round) {
        for (int t = tid; t < w; t += nt) nxt[t] = cur[cur[t]];
        __syncthreads();
        int* tmp = cur; cur = nxt; nxt = tmp;
    }
    // cur[t] = f(t).  prev from the sorted keys: key index i holds (p, t).
    for (int i = tid; i < w; i += nt) {
        const int k = s.key[i];
        const int t = k & 1023, q = k >> 10;
        const int prv = (i > 0 && (s.key[i - 1] >> 10) == q) ? (s.key[i - 1] & 1023) : -1;
        const bool last = (i + 1 >= w) || ((s.key[i + 1] >> 10) != q);
        const int src = (q == t) ? cur[t] : (prv >= 0 ? cur[prv] : q);
        if (src != t) {
            const int slot = atomicAdd(&s.count_top, 1);
            moves[2 + 2 * slot] = t;
            moves[3 + 2 * slot] = src;
        }
        if (q >= w && last) {
            const int slot = atomicAdd(&s.count_extra, 1);
            moves[kMovesExtra + 2 * slot] = q;
            moves[kMovesExtra + 1 + 2 * slot] = cur[t];
        }
    }
    __syncthreads();
    if (tid == 0) { moves[0] = s.count_top; moves[1] = s.count_extra; }
}

}  // namespace lu
