// Cholesky panel: the factorization of one column block of a symmetric
// positive definite matrix, A = L L^T on the lower triangle.  Cholesky fits
// the blocked skeleton of the paper (Sec. 3.1): per iteration the panel (the
// diagonal block and the column block below it) is factored and the trailing
// matrix receives a symmetric rank-b update; the look-ahead reorganization of
// Sec. 4 applies unchanged, with no pivoting and so no row interchanges.
//
// One persistent launch of P work-groups (256 threads each) factors the m x w
// panel (rows relative to the panel's diagonal, m >= w), in blocks of 16
// columns.  Thread t of work-group g owns panel rows g*256 + t + s*256*P
// (s < ROWS, 2 or 4: the launch has at least m / (256 ROWS) work-groups).
// For each block [cb, cb+16):
//   every work-group reads the block's 16 x 16 diagonal part and factors it in
//   LDS (one wave; all groups compute the same values);
//   each thread solves its rows below the diagonal part against it
//   (x <- x L_bb^-T, forward substitution, true division);
//   device-wide barrier (the solved rows of the panel's own diagonal region
//   are the other operand of the next step, and no group still reads the
//   diagonal part, which group 0 now overwrites with the factor);
//   each thread updates its rows of the panel columns to the right of the
//   block, lower triangle only (A[i,c] -= sum_k L[i,cb+k] L[c,cb+k], c <= i);
//   device-wide barrier (the next block's diagonal part was written by
//   whichever group owns it).
// Every element receives its updates in the order of the unblocked algorithm
// (column k = 0, 1, ... of the whole matrix), each as a separate multiply and
// subtract, so the panel's result does not depend on P.
//
// Every access to the panel is a relaxed device-scope atomic (common.hpp:
// it bypasses the per-CU and per-XCD caches), and the barriers drain and
// count without cache write-back or invalidate, as in the LU panel: at device
// scope those act on a whole XCD's L2 and stall the update running beside the
// panel, and they left plain stores of one work-group in its XCD's L2 until
// another work-group's maintenance ran.
#include "common.hpp"
#include "kernels.hpp"

namespace lu {

namespace {

constexpr int kCholThreads = 256;
constexpr int kCholNB = 16;
constexpr int kCholMaxW = 512;
constexpr int kChunkCols = 8;     // columns per pass of the in-panel update (wider passes spill)

template <typename T, int kCholRows>
__global__ __launch_bounds__(kCholThreads) void chol_panel_kernel(CholPanelArgs<T> a) {
    __shared__ T D[kCholNB][kCholNB + 1];                  // the block's factored diagonal part
    __shared__ T UtT[kCholNB][kCholMaxW];                  // L rows of the panel's diagonal region, transposed
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    const int g = blockIdx.x;
    const int P = gridDim.x;
    const int m = a.m, w = a.w;
    const long long lda = a.lda;
    T* __restrict__ A = a.A;
    constexpr int S = __HIP_MEMORY_SCOPE_AGENT;
    unsigned epoch = 0;
    // the next launch's barrier counter (its previous user has finished)
    if (g == 0 && tid == 0 && a.sync_next) xstore_s<S>(a.sync_next, 0u);
    const int stride = kCholThreads * P;
    constexpr int kChunk = kCholRows <= 2 ? kChunkCols : kChunkCols / 2;   // columns per pass of the in-panel update
    constexpr int kDepth = kCholRows <= 2 ? 4 : 2;          // chunks in flight (as registers allow)

    for (int cb = 0; cb < w; cb += kCholNB) {
        const int nbw = min(kCholNB, w - cb);
        // 1. the diagonal part, factored in LDS by wave 0
        for (int e = tid; e < kCholNB * kCholNB; e += kCholThreads) {
            const int r = e % kCholNB, c = e / kCholNB;
            D[r][c] = (r < nbw && c <= r) ? cload<S>(A + (cb + r) + (long long)(cb + c) * lda) : T(0);
        }
        if (tid == 0) s_bad = 0;
        __syncthreads();
        if (tid < kWave) {
            const int i = tid;           // lane i owns row i of the diagonal part
            for (int j = 0; j < nbw; ++j) {
                const T d = D[j][j];
                const T r = sqrt(d);
                if (!(d > T(0)) && i == 0 && s_bad == 0) s_bad = j + 1;
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                if (i == j) D[j][j] = r;
                if (i > j && i < nbw) D[i][j] = D[i][j] / r;            // column j of L
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                if (i > j && i < nbw) {
                    const T lij = D[i][j];
                    for (int c = j + 1; c <= i; ++c) D[i][c] = D[i][c] - lij * D[c][j];
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            }
        }
        __syncthreads();
        // 2. rows below the diagonal part: x <- x L_bb^-T for all of this
        //    thread's rows at once; the solved rows stay in registers as the
        //    left operand of step 3
        const int right0 = cb + nbw;
        const int row0 = right0 + g * kCholThreads + tid;
        T x[kCholRows][kCholNB];
#pragma unroll
        for (int r = 0; r < kCholRows; ++r) {
            const int i = row0 + r * stride;
            const int ic = min(i, m - 1);              // clamped: unconditional loads
#pragma unroll
            for (int c = 0; c < kCholNB; ++c) {
                const T v = cload<S>(A + ic + (long long)(cb + min(c, nbw - 1)) * lda);
                x[r][c] = (i < m && c < nbw) ? v : T(0);
            }
        }
#pragma unroll
        for (int c = 0; c < kCholNB; ++c) {
            if (c < nbw) {
                const T dcc = D[c][c];
#pragma unroll
                for (int k = 0; k < c; ++k) {
                    const T dck = D[c][k];
#pragma unroll
                    for (int r = 0; r < kCholRows; ++r) x[r][c] = x[r][c] - x[r][k] * dck;
                }
#pragma unroll
                for (int r = 0; r < kCholRows; ++r) x[r][c] = x[r][c] / dcc;
            }
        }
#pragma unroll
        for (int r = 0; r < kCholRows; ++r) {
            const int i = row0 + r * stride;
            if (i < m) {
#pragma unroll
                for (int c = 0; c < kCholNB; ++c)
                    if (c < nbw) cstore<S>(A + i + (long long)(cb + c) * lda, x[r][c]);
            }
        }
        // every group has read the diagonal part (step 1) before group 0
        // overwrites it with the factor
        if (grid_barrier_nofence(a.sync, a.sync + 1, ++epoch, a.spin_limit, P)) return;
        if (g == 0) {
            for (int e = tid; e < kCholNB * kCholNB; e += kCholThreads) {
                const int r = e % kCholNB, c = e / kCholNB;
                if (r < nbw && c <= r) cstore<S>(A + (cb + r) + (long long)(cb + c) * lda, D[r][c]);
            }
            if (tid == 0 && s_bad != 0 && a.info) atomicCAS(a.info, 0, a.info_col_base + cb + s_bad);
        }
        if (right0 >= w) break;
        // 3. the panel columns right of the block, lower triangle, kChunk
        //    columns at a time.  Every load is unconditional (clamped
        //    address): a conditional load compiles to a branch, and each one
        //    then waits for its round trip before the next is issued.
        {
            const int wr = (w - right0 + kChunk - 1) / kChunk * kChunk;     // zero past w: whole chunks
            const int ne = wr * kCholNB;
            constexpr int kBatch = 16;                                      // loads in flight per thread
            for (int e0 = 0; e0 < ne; e0 += kBatch * kCholThreads) {
                T t[kBatch];
#pragma unroll
                for (int q = 0; q < kBatch; ++q) {
                    const int e = min(e0 + q * kCholThreads + tid, ne - 1);
                    const int c = e % wr, k = e / wr;
                    t[q] = cload<S>(A + min(right0 + c, w - 1) + (long long)(cb + min(k, nbw - 1)) * lda);
                }
#pragma unroll
                for (int q = 0; q < kBatch; ++q) {
                    const int e = e0 + q * kCholThreads + tid;
                    const int c = e % wr, k = e / wr;
                    if (e < ne) UtT[k][c] = (k < nbw && right0 + c < w) ? t[q] : T(0);
                }
            }
        }
        __syncthreads();
        // Chunks of this thread's rows, kDepth of them in flight: a chunk is
        // loaded kDepth chunks ahead of its arithmetic.  Elements outside the
        // lower triangle or the panel are loaded from a clamped address,
        // updated and never stored.
        auto load_chunk = [&](int c0, T (&v)[kCholRows][kChunk]) {
#pragma unroll
            for (int r = 0; r < kCholRows; ++r) {
                const int ic = min(row0 + r * stride, m - 1);
#pragma unroll
                for (int cc = 0; cc < kChunk; ++cc) v[r][cc] = cload<S>(A + ic + (long long)min(c0 + cc, w - 1) * lda);
            }
        };
        const int nch = (w - right0 + kChunk - 1) / kChunk;
        T v[kDepth][kCholRows][kChunk];
#pragma unroll
        for (int d = 0; d < kDepth; ++d)
            if (d < nch) load_chunk(right0 + d * kChunk, v[d]);
        for (int ch = 0; ch < nch; ch += kDepth) {
#pragma unroll
            for (int d = 0; d < kDepth; ++d) {
                const int q = ch + d;
                if (q >= nch) break;
                const int c0 = right0 + q * kChunk;
#pragma unroll
                for (int cc = 0; cc < kChunk; ++cc) {
#pragma unroll
                    for (int k = 0; k < kCholNB; ++k) {
                        const T u = UtT[k][c0 - right0 + cc];
#pragma unroll
                        for (int r = 0; r < kCholRows; ++r) v[d][r][cc] = v[d][r][cc] - x[r][k] * u;
                    }
                }
#pragma unroll
                for (int r = 0; r < kCholRows; ++r) {
                    const int i = row0 + r * stride;
#pragma unroll
                    for (int cc = 0; cc < kChunk; ++cc) {
                        const int c = c0 + cc;
                        if (i < m && c < w && c <= i) cstore<S>(A + i + (long long)c * lda, v[d][r][cc]);
                    }
                }
                if (q + kDepth < nch) load_chunk(c0 + kDepth * kChunk, v[d]);
            }
        }
        if (grid_barrier_nofence(a.sync, a.sync + 1, ++epoch, a.spin_limit, P)) return;
    }
}

}  // namespace

template <typename T>
int launch_chol_panel(const CholPanelArgs<T>& args, int wgs, hipStream_t stream) {
    if (args.w < 1 || args.w > kCholMaxW || args.m < args.w || wgs < 1) return -1;
    const long long per = (long long)wgs * kCholThreads;     // rows per thread-slot sweep
    if (per * 2 >= args.m)
        hipLaunchKernelGGL((chol_panel_kernel<T, 2>), dim3(wgs), dim3(kCholThreads), 0, stream, args);
    else if (per * 4 >= args.m)
        hipLaunchKernelGGL((chol_panel_kernel<T, 4>), dim3(wgs), dim3(kCholThreads), 0, stream, args);
    else
        return -1;                                            // more than 4 rows per thread
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template int launch_chol_panel<double>(const CholPanelArgs<double>&, int, hipStream_t);

}  // namespace lu
