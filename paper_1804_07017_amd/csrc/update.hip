// Row interchanges and the U12 triangular solve of one elimination step
// (paper Sec. 3.4: laswp and trsm of getrf; Sec. 3.5: RL2 of LU_blk,
// A12 := trilu(A11)^-1 A12, trilu = the unit lower triangle).
//
// swap_trsm_kernel: one work-group per BN columns of the trailing block.
//   1. gather: the w top rows of its columns into LDS, with the panel's
//      composed interchanges applied (rows that received another row's data
//      read it from that row); the extra rows (interchange targets below the
//      top w rows) are read too and written back only after every read of
//      the work-group's columns is done;
//   2. forward substitution with the unit lower w x w block L11, staged in
//      LDS by column chunks;
//   3. the U12 rows go back to the matrix (and, in the mixed-precision mode,
//      to a half-precision copy with one power-of-two scale per column).
// lswap_kernel: the same interchanges on finished columns left of the panel.
#include "common.hpp"
#include "kernels.hpp"

namespace lu {

namespace {

constexpr int kThreads = 256;

template <typename T> struct HalfOf { typedef _Float16 type; };

// largest power of two p with p * amax < 2^15 (so scaled values stay below
// the FP16 maximum after rounding); 1 for amax == 0 or non-finite amax
__device__ __forceinline__ float pow2_scale(float amax) {
    if (!(amax > 0.f) || !(amax < 3.0e38f)) return 1.f;
    int e;
    frexpf(amax, &e);                    // amax = f * 2^e, f in [0.5, 1)
    return ldexpf(1.f, 15 - e);          // amax * 2^(15-e) in [2^14, 2^15)
}

template <typename T, typename H>
__global__ __launch_bounds__(kThreads) void swap_trsm_kernel(SwapTrsmArgs<T, H> a) {
    extern __shared__ unsigned char smem_raw[];
    const int w = a.w, BN = a.bn;
    const int ldx = BN + 1;
    T* X = reinterpret_cast<T*>(smem_raw);              // [w][BN+1] the top rows
    T* V = X + (size_t)w * ldx;                         // [w][BN]  extra-row values, later L chunks

    const int tid = threadIdx.x;
    const int c_base = a.c0 + blockIdx.x * BN;
    const int nc = min(BN, a.c1 - c_base);
    const long long lda = a.lda;
    T* __restrict__ Atop = a.A + a.r0;                  // row r0 of column 0
    __shared__ int mv[2 * 2 * kMovesMaxW];   // (dst, src): top moves, then extra moves
    const int ntop = a.moves[0], nex = a.moves[1];
    for (int s = tid; s < ntop; s += kThreads) { mv[2 * s] = a.moves[2 + 2 * s]; mv[2 * s + 1] = a.moves[3 + 2 * s]; }
    for (int s = tid; s < nex; s += kThreads) {
        mv[2 * (ntop + s)] = a.moves[kMovesExtra + 2 * s];
        mv[2 * (ntop + s) + 1] = a.moves[kMovesExtra + 1 + 2 * s];
    }

    // 1. gather (reads only), batched so that many loads are in flight
    constexpr int kBatch = 8;
    for (int e0 = tid; e0 < w * BN; e0 += kThreads * kBatch) {
        T v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = e0 + u * kThreads;
            const int t = e % w, c = e / w;
            v[u] = (e < w * BN && c < nc) ? Atop[t + (long long)(c_base + c) * lda] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = e0 + u * kThreads;
            if (e < w * BN) X[(e % w) * ldx + e / w] = v[u];
        }
    }
    __syncthreads();
    const int cnt = ntop + nex;
    for (int e0 = tid; e0 < cnt * BN; e0 += kThreads * kBatch) {
        T v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = e0 + u * kThreads;
            const int s = e / BN, c = e % BN;
            v[u] = (e < cnt * BN && c < nc) ? Atop[mv[2 * s + 1] + (long long)(c_base + c) * lda] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = e0 + u * kThreads;
            if (e < cnt * BN) {
                const int s = e / BN, c = e % BN;
                if (s < ntop) X[mv[2 * s] * ldx + c] = v[u];
                else V[(s - ntop) * BN + c] = v[u];
            }
        }
    }
    __syncthreads();
    // scatter of the extra rows, after every read of these columns
    for (int e = tid; e < nex * BN; e += kThreads) {
        const int s = e / BN, c = e % BN;
        if (c < nc) Atop[mv[2 * (ntop + s)] + (long long)(c_base + c) * lda] = V[s * BN + c];
    }
    __syncthreads();

    // 2. forward substitution with unit-lower L11 in blocks of KB rows:
    //    (a) the KB x KB diagonal block, one thread per column;
    //    (b) the rows below, X[i] -= L[i, blk] X[blk], all threads.
    //    L11's block columns are staged into V (w x BN values >= (w-k0) x KB);
    //    the next block's columns are loaded into registers while the current
    //    block is being solved, so their latency is hidden.
    constexpr int kPre = 16;                      // staged values per thread per block
    // KB <= BN (V capacity) and w*KB <= kPre*256 (register prefetch capacity)
    const int KB = min(min(BN, 16), (kPre * kThreads) / w);
    const T* __restrict__ L = a.A + a.r0 + (long long)a.r0 * lda;   // L11 at (r0, r0)
    T pre[kPre];
    auto fetch = [&](int k0) {
        const int rows = w - k0, kb = min(KB, w - k0);
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int e = tid + u * kThreads;
            const int i = e % rows, s = e / rows;
            const bool ok = e < rows * kb;
            pre[u] = L[(k0 + (ok ? i : 0)) + (long long)(k0 + (ok ? s : 0)) * lda];
        }
    };
    auto stage = [&](int k0) {
        const int rows = w - k0, kb = min(KB, w - k0);
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int e = tid + u * kThreads;
            if (e < rows * kb) V[(e % rows) * KB + e / rows] = pre[u];
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < w; k0 += KB) {
        const int kb = min(KB, w - k0);
        const int rows = w - k0;
        stage(k0);
        __syncthreads();
        if (k0 + KB < w) fetch(k0 + KB);
        if (tid < BN) {
            const int c = tid;
            for (int s = 0; s < kb; ++s) {
                const T xs = X[(k0 + s) * ldx + c];
                for (int r = s + 1; r < kb; ++r) X[(k0 + r) * ldx + c] -= V[r * KB + s] * xs;
            }
        }
        __syncthreads();
        const int below = rows - kb;
        for (int e = tid; e < below * BN; e += kThreads) {
            const int ii = kb + e / BN, c = e % BN;
            T acc = X[(k0 + ii) * ldx + c];
#pragma unroll 4
            for (int s = 0; s < kb; ++s) acc -= V[ii * KB + s] * X[(k0 + s) * ldx + c];
            X[(k0 + ii) * ldx + c] = acc;
        }
        __syncthreads();
    }
    // 3. U12 back to the matrix (and the scaled half copy)
    for (int e = tid; e < w * BN; e += kThreads) {
        const int t = e % w, c = e / w;
        if (c < nc) Atop[t + (long long)(c_base + c) * lda] = X[t * ldx + c];
    }
    if (a.uh) {
        __shared__ float s_scale[64];
        if (tid < BN) {
            float amax = 0.f;
            for (int t = 0; t < w; ++t) amax = fmaxf(amax, fabsf((float)X[t * ldx + tid]));
            const float sc = pow2_scale(amax);
            s_scale[tid] = sc;
            if (tid < nc) a.cs[c_base + tid] = 1.f / sc;
        }
        __syncthreads();
        for (int e = tid; e < w * BN; e += kThreads) {
            const int t = e % w, c = e / w;
            if (c < nc) a.uh[(long long)(c_base + c) * a.lduh + t] = (H)((float)X[t * ldx + c] * s_scale[c]);
        }
    }
}

// Interchanges only, on columns [c0, c1): all reads of a column before its writes.
template <typename T>
__global__ __launch_bounds__(kThreads) void lswap_kernel(T* A, long long lda, int r0, const int* moves, int c0,
                                                         int c1, int cols_per_wg) {
    __shared__ int mv[2 * 2 * kMovesMaxW];   // (dst, src) pairs, top then extra
    const int tid = threadIdx.x;
    const int ntop = moves[0], nex = moves[1];
    const int cnt = ntop + nex;
    for (int s = tid; s < ntop; s += kThreads) { mv[2 * s] = moves[2 + 2 * s]; mv[2 * s + 1] = moves[3 + 2 * s]; }
    for (int s = tid; s < nex; s += kThreads) {
        mv[2 * (ntop + s)] = moves[kMovesExtra + 2 * s];
        mv[2 * (ntop + s) + 1] = moves[kMovesExtra + 1 + 2 * s];
    }
    __syncthreads();
    constexpr int kPer = (2 * kMovesMaxW + kThreads - 1) / kThreads;
    const int cb = c0 + blockIdx.x * cols_per_wg;
    for (int c = cb; c < min(c1, cb + cols_per_wg); ++c) {
        T* col = A + r0 + (long long)c * lda;
        T v[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int s = tid + u * kThreads;
            if (s < cnt) v[u] = col[mv[2 * s + 1]];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int s = tid + u * kThreads;
            if (s < cnt) col[mv[2 * s]] = v[u];
        }
        __syncthreads();
    }
}

// Interchange moves of a standalone run of pivots (relative rows).
// A pivot outside [t, m) is not a legal interchange and is treated as none.
__global__ __launch_bounds__(kThreads) void moves_kernel(const int* ipiv_rel, int w, int m, int* moves) {
    __shared__ int p[kMovesMaxW];
    __shared__ MovesScratch ms;
    for (int t = threadIdx.x; t < w; t += kThreads) {
        const int q = ipiv_rel[t];
        p[t] = (q >= t && q < m) ? q : t;
    }
    __syncthreads();
    compose_moves(p, w, moves, ms);
}

// Per-chunk moves for a long pivot vector: chunk c covers steps
// [c*W, min(n, (c+1)*W)), rows relative to c*W.  moves stride = kMovesLen.
__global__ __launch_bounds__(kThreads) void chunk_moves_kernel(const int* ipiv, int n, int W, int* moves) {
    __shared__ int p[kMovesMaxW];
    __shared__ MovesScratch ms;
    const int c = blockIdx.x;
    const int base = c * W;
    const int w = min(W, n - base);
    for (int t = threadIdx.x; t < w; t += kThreads) {
        const int q = ipiv[base + t] - base;          // illegal pivots are treated as no interchange
        p[t] = (q >= t && q < n - base) ? q : t;
    }
    __syncthreads();
    compose_moves(p, w, moves + (size_t)c * kMovesLen, ms);
}

// A21 rows -> half precision, row-major with one power-of-two scale per row:
// Lh[i][kk] = A[i][kk] * 2^s_i, rs[i] = 2^-s_i.  64 rows per work-group.
template <typename H>
__global__ __launch_bounds__(kThreads) void l21_half_kernel(const float* A, long long lda, int m, int w, H* Lh,
                                                            long long ldh, float* rs, int rows) {
    extern __shared__ unsigned char smem_raw[];
    float* T = reinterpret_cast<float*>(smem_raw);   // [rows][w+1]
    __shared__ float s_sc[64];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * rows;
    const int nr = min(rows, m - r0);
    const int ldt = w + 1;
    for (int e = tid; e < rows * w; e += kThreads) {
        const int r = e % rows, k = e / rows;
        T[r * ldt + k] = (r < nr) ? A[(r0 + r) + (long long)k * lda] : 0.f;
    }
    __syncthreads();
    if (tid < rows) {
        float amax = 0.f;
        for (int k = 0; k < w; ++k) amax = fmaxf(amax, fabsf(T[tid * ldt + k]));
        const float sc = pow2_scale(amax);
        s_sc[tid] = sc;
        if (tid < nr) rs[r0 + tid] = 1.f / sc;
    }
    __syncthreads();
    for (int e = tid; e < rows * w; e += kThreads) {
        const int r = e / w, k = e % w;
        if (r < nr) Lh[(long long)(r0 + r) * ldh + k] = (H)(T[r * ldt + k] * s_sc[r]);
    }
}

// Columns of a column-major k x n block -> half precision, k contiguous, one
// power-of-two scale per column: Uh[j*ldh + kk] = B[kk + j*ldb] * 2^s_j, cs[j] = 2^-s_j.
template <typename H>
__global__ __launch_bounds__(64) void cols_half_kernel(const float* B, long long ldb, int k, int n, H* Uh,
                                                       long long ldh, float* cs) {
    const int j = blockIdx.x;
    const int l = threadIdx.x;
    const float* col = B + (long long)j * ldb;
    float amax = 0.f;
    for (int kk = l; kk < k; kk += 64) amax = fmaxf(amax, fabsf(col[kk]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 64));
    const float sc = pow2_scale(amax);
    if (l == 0) cs[j] = 1.f / sc;
    for (int kk = l; kk < k; kk += 64) Uh[(long long)j * ldh + kk] = (H)(col[kk] * sc);
}

}  // namespace

template <typename H>
int launch_cols_half(const float* B, long long ldb, int k, int n, H* Uh, long long ldh, float* cs,
                     hipStream_t stream) {
    if (n <= 0 || k <= 0) return 0;
    hipLaunchKernelGGL((cols_half_kernel<H>), dim3(n), dim3(64), 0, stream, B, ldb, k, n, Uh, ldh, cs);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_cols_half<_Float16>(const float*, long long, int, int, _Float16*, long long, float*, hipStream_t);
template int launch_cols_half<__bf16>(const float*, long long, int, int, __bf16*, long long, float*, hipStream_t);

template <typename T, typename H>
int launch_swap_trsm(const SwapTrsmArgs<T, H>& args0, hipStream_t stream) {
    SwapTrsmArgs<T, H> args = args0;
    if (args.c1 <= args.c0 || args.w <= 0) return 0;
    // X and V each hold w x BN values: keep them within 64 KiB together
    int bn = (int)(32768 / (sizeof(T) * args.w));
    if (bn > 64) bn = 64;
    if (bn < 1) bn = 1;
    args.bn = bn;
    const size_t smem = (size_t)args.w * (2 * bn + 1) * sizeof(T);
    const int grid = (args.c1 - args.c0 + bn - 1) / bn;
    hipLaunchKernelGGL((swap_trsm_kernel<T, H>), dim3(grid), dim3(kThreads), smem, stream, args);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_lswap(T* A, long long lda, int r0, const int* moves, int c0, int c1, hipStream_t stream) {
    if (c1 <= c0) return 0;
    const int per = 4;
    const int grid = (c1 - c0 + per - 1) / per;
    hipLaunchKernelGGL((lswap_kernel<T>), dim3(grid), dim3(kThreads), 0, stream, A, lda, r0, moves, c0, c1, per);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_moves(const int* ipiv_rel, int w, int m, int* moves, hipStream_t stream) {
    hipLaunchKernelGGL(moves_kernel, dim3(1), dim3(kThreads), 0, stream, ipiv_rel, w, m, moves);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_chunk_moves(const int* ipiv, int n, int W, int* moves, hipStream_t stream) {
    if (n <= 0) return 0;
    const int chunks = (n + W - 1) / W;
    hipLaunchKernelGGL(chunk_moves_kernel, dim3(chunks), dim3(kThreads), 0, stream, ipiv, n, W, moves);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename H>
int launch_l21_half(const float* A, long long lda, int m, int w, H* Lh, long long ldh, float* rs,
                    hipStream_t stream) {
    if (m <= 0 || w <= 0) return 0;
    const int rows = w <= 128 ? 64 : (w <= 256 ? 32 : 16);
    const size_t smem = sizeof(float) * rows * (size_t)(w + 1);
    hipLaunchKernelGGL((l21_half_kernel<H>), dim3((m + rows - 1) / rows), dim3(kThreads), smem, stream, A, lda, m, w,
                       Lh, ldh, rs, rows);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_swap_trsm<double, _Float16>(const SwapTrsmArgs<double, _Float16>&, hipStream_t);
template int launch_swap_trsm<float, _Float16>(const SwapTrsmArgs<float, _Float16>&, hipStream_t);
template int launch_swap_trsm<float, __bf16>(const SwapTrsmArgs<float, __bf16>&, hipStream_t);
template int launch_lswap<double>(double*, long long, int, const int*, int, int, hipStream_t);
template int launch_lswap<float>(float*, long long, int, const int*, int, int, hipStream_t);
template int launch_l21_half<_Float16>(const float*, long long, int, int, _Float16*, long long, float*,
                                       hipStream_t);
template int launch_l21_half<__bf16>(const float*, long long, int, int, __bf16*, long long, float*, hipStream_t);

}  // namespace lu
