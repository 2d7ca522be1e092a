// Trailing-matrix update, RL3 of LU_blk (paper Sec. 3.5): C -= A * B with
// A = A21 (m x k), B = A12 (k x n) and k = the block size b.  This is where
// the flops are (Sec. 3.2: the panel width is kept small so that most work
// is this compute-bound update).
//
// gfx950 MFMA tiles, 256 threads = 4 waves per work-group, 128 x 128 output
// tile per work-group (64 x 64 per wave = 4 x 4 MFMA 16x16 blocks).  The
// operands are staged through LDS, double-buffered, one k-tile ahead.
//
// Operand roles are swapped inside the MFMA: the instruction's first operand
// takes B (so its 16 output rows run along C's columns) and its second takes
// -A (output columns along C's rows).  A lane then holds 16 consecutive ROWS
// of one C column, which is what column-major C wants for coalesced loads
// and stores.  For FP64/FP32 the accumulators start from C itself, so the
// update is C + sum_k (-a_ik) b_kj accumulated in the matrix core.
//
// Element (i,j) of C sees the same sequence of operations whatever the tile
// it falls in, so splitting the update into several launches (the look-ahead
// schedule does) leaves the result bit-identical.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace lu {

namespace {

constexpr int kBM = 128, kBN = 128, kThreads = 256;

// Map the linear work-group id to a (tile_m, tile_n) pair.  Work-groups are
// dealt to the 8 XCDs round-robin; this remap gives each XCD a contiguous
// chunk of the tile order, and the order walks kGroupM tile-rows down before
// moving to the next tile column, so that the A rows and B columns of the
// tiles an XCD runs at the same time stay in its L2.
//
// A triangular update (LOW below) keeps the plain order instead: its empty
// tiles sit at the top of the tile order, and dealing contiguous chunks to
// the XCDs would leave the first XCDs nearly idle; in plain order every XCD
// takes every 8th tile, a fair share of the full ones.
constexpr int kGroupM = 8;
// Tile order: linear tile L walks kGroupM tile-rows down before moving to the
// next tile column.
__device__ __forceinline__ void tile_coords(int L, int tiles_m, int tiles_n, int& tm, int& tn) {
    const int grp = kGroupM * tiles_n;
    const int gi = L / grp, r = L % grp;
    const int m0 = gi * kGroupM;
    const int gh = min(kGroupM, tiles_m - m0);
    tm = m0 + r % gh;
    tn = r / gh;
}
// One tile per work-group: work-group b runs on XCD b % 8, so b is remapped
// to give each XCD a contiguous chunk of the tile order.
__device__ __forceinline__ int tile_of_block(int nt, bool xcd_chunks) {
    int bid = blockIdx.x;
    const int per = nt / 8;
    if (xcd_chunks && per > 0 && bid < per * 8) bid = (bid % 8) * per + bid / 8;
    return bid;
}

// The tile body.  TB: B is given transposed (element (k, j) at B[j + k*ldb]),
// as in the symmetric update A22 -= L21 L21^T where both operands are the
// same column block.  LOW: only C's lower triangle is updated -- element
// (i, j) of C when i + diag >= j -- tiles wholly above it are skipped and
// tiles across it store only their lower part.
template <typename T, int BK, bool TB, bool LOW, bool ZERO = false, int BM = kBM>
__device__ __forceinline__ void gemm_tile(int L, int M, int N, int K, const T* __restrict__ A, int lda,
                                          const T* __restrict__ B, int ldb, T* __restrict__ C, int ldc,
                                          int diag) {
    typedef typename Acc<T>::type V4;
    constexpr int PA = 2, PB = 1;
    constexpr int WTM = BM / 2, RB = WTM / 16;      // rows per wave and 16-row blocks per wave
    __shared__ T As[2][BK][BM + PA];
    __shared__ T Bs[2][kBN][BK + PB];

    const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + kBN - 1) / kBN;
    int tm, tn;
    tile_coords(L, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * kBN;
    if constexpr (LOW) {
        if (m0 + BM - 1 + diag < n0) return;          // the whole tile lies above the diagonal
    }
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int l16 = lane % 16, lg = lane / 16;
    const int wm = wave % 2, wn = wave / 2;

    // Tiles inside the matrix (all but the last tile row and column) take a
    // branch-free path: no per-element bounds checks, B read two k at a time.
    const bool interior = m0 + BM <= M && n0 + kBN <= N;
    const bool vecb = !TB && interior && (reinterpret_cast<unsigned long long>(B) % (2 * sizeof(T))) == 0 &&
                      (ldb % 2) == 0;
    // LOW: tiles wholly below the diagonal store everything
    const bool full = !LOW || m0 + diag >= n0 + kBN - 1;

    // accumulators start from C (ZERO: from 0, C is only written)
    V4 acc[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        if constexpr (ZERO) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[rb][cb][r] = T(0);
            continue;
        }
        const int row = m0 + wm * WTM + rb * 16 + l16;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int col = n0 + wn * 64 + cb * 16 + Acc<T>::col(lg, r);
                if (interior) acc[rb][cb][r] = C[row + (long long)col * ldc];
                else acc[rb][cb][r] = (row < M && col < N) ? C[row + (long long)col * ldc] : T(0);
            }
        }
    }

    // global -> register staging
    constexpr int AL = BK * BM / kThreads;    // A elements per thread
    constexpr int BL = BK * kBN / kThreads;   // B elements per thread
    T ra[AL], rbv[BL];
    const int a_row = tid % BM, a_k0 = tid / BM;                // A: rows contiguous
    constexpr int AKS = kThreads / BM;
    const int b_col = tid / (kThreads / kBN), b_kh = tid % (kThreads / kBN);   // B: k contiguous
    constexpr int BKS = BK / (kThreads / kBN);
    const int t_col = tid % kBN, t_k0 = tid / kBN;                               // B^T: j contiguous
    constexpr int TKS = kThreads / kBN;

    static_assert(BKS % 2 == 0, "B is read two k at a time");
    typedef T T2 __attribute__((ext_vector_type(2)));
    auto load = [&](int k0) {
        if (interior && k0 + BK <= K) {
#pragma unroll
            for (int r = 0; r < AL; ++r) ra[r] = A[m0 + a_row + (long long)(k0 + a_k0 + AKS * r) * lda];
            if constexpr (TB) {
#pragma unroll
                for (int e = 0; e < BL; ++e) rbv[e] = B[n0 + t_col + (long long)(k0 + t_k0 + TKS * e) * ldb];
                return;
            }
            const T* bp = B + k0 + b_kh * BKS + (long long)(n0 + b_col) * ldb;
            if (vecb) {
#pragma unroll
                for (int e = 0; e < BL; e += 2) {
                    const T2 v = *reinterpret_cast<const T2*>(bp + e);
                    rbv[e] = v.x;
                    rbv[e + 1] = v.y;
                }
            } else {
#pragma unroll
                for (int e = 0; e < BL; ++e) rbv[e] = bp[e];
            }
            return;
        }
#pragma unroll
        for (int r = 0; r < AL; ++r) {
            const int kk = a_k0 + AKS * r;
            const int gr = m0 + a_row, gk = k0 + kk;
            ra[r] = (gr < M && gk < K) ? A[gr + (long long)gk * lda] : T(0);
        }
#pragma unroll
        for (int e = 0; e < BL; ++e) {
            if constexpr (TB) {
                const int gc = n0 + t_col, gk = k0 + t_k0 + TKS * e;
                rbv[e] = (gc < N && gk < K) ? B[gc + (long long)gk * ldb] : T(0);
            } else {
                const int kk = b_kh * BKS + e;
                const int gc = n0 + b_col, gk = k0 + kk;
                rbv[e] = (gc < N && gk < K) ? B[gk + (long long)gc * ldb] : T(0);
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < AL; ++r) As[buf][a_k0 + AKS * r][a_row] = -ra[r];
#pragma unroll
        for (int e = 0; e < BL; ++e) {
            if constexpr (TB) Bs[buf][t_col][t_k0 + TKS * e] = rbv[e];
            else Bs[buf][b_col][b_kh * BKS + e] = rbv[e];
        }
    };

    const int nk = (K + BK - 1) / BK;
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            T af[RB], bf[4];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) af[rb] = As[cur][ks * 4 + lg][wm * WTM + rb * 16 + l16];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) bf[cb] = Bs[cur][wn * 64 + cb * 16 + l16][ks * 4 + lg];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = mfma(bf[cb], af[rb], acc[rb][cb]);
        }
        if (kt + 1 < nk) store(cur ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int row = m0 + wm * WTM + rb * 16 + l16;
        if (interior || row < M) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int col = n0 + wn * 64 + cb * 16 + Acc<T>::col(lg, r);
                    if ((interior || col < N) && (full || row + diag >= col))
                        C[row + (long long)col * ldc] = acc[rb][cb][r];
                }
            }
        }
    }
}

// The LU's trailing update runs 64 x 128 tiles (each wave 32 x 64), three
// work-groups per CU: measured faster than 128 x 128 at two per CU for the
// short k of a panel (FP64, 32768^2 x 256: 9.6 against 10.3 ms).  Element
// (i, j) sees the same MFMA sequence in either tile shape.
constexpr int kLuBM = 64;
template <typename T, int BK>
__global__ __launch_bounds__(kThreads, 3) void gemm_nn_sub(int M, int N, int K, const T* __restrict__ A,
                                                            int lda, const T* __restrict__ B, int ldb,
                                                            T* __restrict__ C, int ldc) {
    const int nt = ((M + kLuBM - 1) / kLuBM) * ((N + kBN - 1) / kBN);
    gemm_tile<T, BK, false, false, false, kLuBM>(tile_of_block(nt, true), M, N, K, A, lda, B, ldb, C, ldc, 0);
}

// Tile claiming for a launch beside a panel that holds XCD 0 (the trailing
// update of the look-ahead).  The work-groups on XCD 0 return at once, so no
// work-group of the launch waits for, or holds, a CU there.  The tile order is
// cut into 7 contiguous chunks with one counter each; a work-group on XCD x
// claims tiles of chunk x - 1 (its XCD's L2 keeps that chunk's operands) and,
// once that is exhausted, of the other chunks.  Every tile is claimed exactly
// once whatever the placement.  The next tile is claimed while the current
// one is computed.  claim[0..7]: counters of this launch; next[0..7]: the next
// such launch's (its stream's previous launch has finished), cleared here.
struct TileClaim {
    unsigned* ctr;
    unsigned* next;
    int nt, chunk, home;
    __device__ __forceinline__ int get() const {      // one thread; -1 when none is left
        for (int v = 0; v < 7; ++v) {
            const int c = (home + v) % 7;
            const int lo = c * chunk, len = min(nt, lo + chunk) - lo;
            if (len <= 0) continue;
            if ((int)xload(ctr + c) >= len) continue;
            const int i = (int)atomicAdd(ctr + c, 1u);
            if (i < len) return lo + i;
        }
        return -1;
    }
};

template <typename Body>
__device__ __forceinline__ void claimed_tiles(unsigned* ctr, unsigned* next, int nt, Body body) {
    __shared__ int s_tile;
    if (blockIdx.x == 0 && threadIdx.x < 8) xstore(next + threadIdx.x, 0u);
    const int x = xcd_id();
    if (x == 0) return;
    const TileClaim tc{ctr, next, nt, (nt + 6) / 7, (x - 1) % 7};
    int ahead = threadIdx.x == 0 ? tc.get() : 0;
    for (;;) {
        __syncthreads();                       // every wave has read s_tile of the last round
        if (threadIdx.x == 0) s_tile = ahead;
        __syncthreads();
        const int L = s_tile;
        if (L < 0) break;
        if (threadIdx.x == 0) ahead = tc.get();
        body(L);
    }
}

template <typename T, int BK>
__global__ __launch_bounds__(kThreads, 3) void gemm_nn_sub_x7(int M, int N, int K, const T* __restrict__ A,
                                                               int lda, const T* __restrict__ B, int ldb,
                                                               T* __restrict__ C, int ldc, unsigned* ctr,
                                                               unsigned* next) {
    const int nt = ((M + kLuBM - 1) / kLuBM) * ((N + kBN - 1) / kBN);
    claimed_tiles(ctr, next, nt, [&](int L) {
        gemm_tile<T, BK, false, false, false, kLuBM>(L, M, N, K, A, lda, B, ldb, C, ldc, 0);
    });
}

// The same product for the Householder block updates (QR, band reduction):
// a kernel of its own so that profiles keep the LU's trailing update apart.
template <typename T, int BK>
__global__ __launch_bounds__(kThreads, 2) void gemm_nn_hh(int M, int N, int K, const T* __restrict__ A,
                                                           int lda, const T* __restrict__ B, int ldb,
                                                           T* __restrict__ C, int ldc) {
    const int nt = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
    gemm_tile<T, BK, false, false>(tile_of_block(nt, true), M, N, K, A, lda, B, ldb, C, ldc, 0);
}

// Split-K form for products with a long k range and few output tiles (the
// V^T C product of a Householder block update): the work-groups of slice
// z = blockIdx.y take k in [z*ks, min(K, (z+1)*ks)) and store
// C_z = -A[:, slice] B[slice, :] at C + z*cstride.  Summing the slices in z
// order gives a result that depends on ks only, not on the launch.
template <typename T, int BK>
__global__ __launch_bounds__(kThreads, 2) void gemm_nn_split(int M, int N, int K, int ks,
                                                              const T* __restrict__ A, int lda,
                                                              const T* __restrict__ B, int ldb,
                                                              T* __restrict__ C, int ldc, long long cstride) {
    const int z = blockIdx.y;
    const int k0 = z * ks;
    const int nt = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
    gemm_tile<T, BK, false, false, true>(tile_of_block(nt, true), M, N, min(ks, K - k0), A + (long long)k0 * lda,
                                         lda, B + k0, ldb, C + z * cstride, ldc, 0);
}

// C -= A B^T on the lower triangle of C (the symmetric rank-k update of a
// Cholesky step, B = A's rows of the column block being updated).
template <typename T, int BK>
__global__ __launch_bounds__(kThreads, 2) void syrk_ln_sub(int M, int N, int K, const T* __restrict__ A,
                                                            int lda, const T* __restrict__ B, int ldb,
                                                            T* __restrict__ C, int ldc, int diag) {
    gemm_tile<T, BK, true, true>((int)blockIdx.x, M, N, K, A, lda, B, ldb, C, ldc, diag);
}

// Mixed precision: C (FP32) -= diag(rs) (Ah Bh) diag(cs), Ah = FP16/BF16 rows
// of A21 stored k-contiguous (row-major, leading dimension lda_h), Bh = the
// U12 columns stored k-contiguous (column-major, ldb_h); rs / cs are the
// exact powers of two that undo the operand scaling.  FP32 accumulation in
// v_mfma_f32_16x16x32_{f16,bf16}.
template <typename H> struct HalfOps;
template <> struct HalfOps<_Float16> {
    typedef v8h vec;
    static __device__ __forceinline__ v4f mma(vec a, vec b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct HalfOps<__bf16> {
    typedef v8bf vec;
    static __device__ __forceinline__ v4f mma(vec a, vec b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

template <typename H>
__device__ __forceinline__ void gemm_half_tile(int L, int M, int N, int K, const H* __restrict__ Ah, int lda_h,
                                               const H* __restrict__ Bh, int ldb_h, const float* __restrict__ rs,
                                               const float* __restrict__ cs, float* __restrict__ C, int ldc) {
    typedef typename HalfOps<H>::vec VH;
    constexpr int BK = 64;              // two MFMA k-steps of 32
    constexpr int PADH = 8;             // halves of padding per LDS row
    __shared__ H As[2][kBM][BK + PADH];
    __shared__ H Bs[2][kBN][BK + PADH];

    const int tiles_m = (M + kBM - 1) / kBM, tiles_n = (N + kBN - 1) / kBN;
    int tm, tn;
    tile_coords(L, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * kBM, n0 = tn * kBN;
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int l16 = lane % 16, lg = lane / 16;
    const int wm = wave % 2, wn = wave / 2;

    v4f acc[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = v4f{0.f, 0.f, 0.f, 0.f};
    // The update is bound by C's traffic: its tile and the scales are loaded
    // first, so that they arrive while the matrix cores work.
    v4f cpre[4][4];
    float rsc[4], csc[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int row = m0 + wm * 64 + rb * 16 + l16;
        const bool rok = row < M;
        rsc[rb] = rs[rok ? row : 0];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int col = n0 + wn * 64 + cb * 16 + 4 * lg + r;
                const bool ok = rok && col < N;
                const float v = C[(ok ? row : 0) + (long long)(ok ? col : 0) * ldc];
                cpre[rb][cb][r] = ok ? v : 0.f;
            }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = n0 + wn * 64 + cb * 16 + 4 * lg + r;
            csc[cb][r] = cs[col < N ? col : 0];
        }

    // each thread moves 4 chunks of 8 halves (16 B) for A and for B per k-tile
    const int ld_row = tid / 8 * 1, ld_chunk = tid % 8;      // 32 rows x 8 chunks per pass
    VH ra[4], rb4[4];
    // tiles inside the matrix take a branch-free path (16-byte loads need the
    // k offsets and leading dimensions to be multiples of 8 halves)
    const bool interior = m0 + kBM <= M && n0 + kBN <= N && lda_h % 8 == 0 && ldb_h % 8 == 0 &&
                          (reinterpret_cast<unsigned long long>(Ah) % 16) == 0 &&
                          (reinterpret_cast<unsigned long long>(Bh) % 16) == 0;
    auto load = [&](int k0) {
        if (interior && k0 + BK <= K) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int row = ld_row + 32 * p;
                const int gk = k0 + ld_chunk * 8;
                ra[p] = *reinterpret_cast<const VH*>(Ah + (long long)(m0 + row) * lda_h + gk);
                rb4[p] = *reinterpret_cast<const VH*>(Bh + (long long)(n0 + row) * ldb_h + gk);
            }
            return;
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int row = ld_row + 32 * p;
            const int gk = k0 + ld_chunk * 8;
            const int gr = m0 + row, gc = n0 + row;
            VH za;
#pragma unroll
            for (int e = 0; e < 8; ++e) za[e] = H(0.f);
            ra[p] = za;
            rb4[p] = za;
            if (gr < M) {
                if (gk + 8 <= K) ra[p] = *reinterpret_cast<const VH*>(Ah + (long long)gr * lda_h + gk);
                else for (int e = 0; e < 8; ++e) if (gk + e < K) ra[p][e] = Ah[(long long)gr * lda_h + gk + e];
            }
            if (gc < N) {
                if (gk + 8 <= K) rb4[p] = *reinterpret_cast<const VH*>(Bh + (long long)gc * ldb_h + gk);
                else for (int e = 0; e < 8; ++e) if (gk + e < K) rb4[p][e] = Bh[(long long)gc * ldb_h + gk + e];
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            *reinterpret_cast<VH*>(&As[buf][ld_row + 32 * p][ld_chunk * 8]) = ra[p];
            *reinterpret_cast<VH*>(&Bs[buf][ld_row + 32 * p][ld_chunk * 8]) = rb4[p];
        }
    };
    const int nk = (K + BK - 1) / BK;
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK / 32; ++ks) {
            VH af[4], bf[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
                af[rb] = *reinterpret_cast<const VH*>(&As[cur][wm * 64 + rb * 16 + l16][ks * 32 + lg * 8]);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                bf[cb] = *reinterpret_cast<const VH*>(&Bs[cur][wn * 64 + cb * 16 + l16][ks * 32 + lg * 8]);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = HalfOps<H>::mma(bf[cb], af[rb], acc[rb][cb]);
        }
        if (kt + 1 < nk) store(cur ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int row = m0 + wm * 64 + rb * 16 + l16;
        if (row < M) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int col = n0 + wn * 64 + cb * 16 + 4 * lg + r;
                    if (col < N) C[row + (long long)col * ldc] = cpre[rb][cb][r] - (acc[rb][cb][r] * rsc[rb]) * csc[cb][r];
                }
            }
        }
    }
}


template <typename H>
__global__ __launch_bounds__(kThreads, 2) void gemm_half_sub(int M, int N, int K, const H* __restrict__ Ah,
                                                              int lda_h, const H* __restrict__ Bh, int ldb_h,
                                                              const float* __restrict__ rs,
                                                              const float* __restrict__ cs,
                                                              float* __restrict__ C, int ldc) {
    const int nt = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
    gemm_half_tile<H>(tile_of_block(nt, true), M, N, K, Ah, lda_h, Bh, ldb_h, rs, cs, C, ldc);
}

// XCD 0 left free, tiles claimed as in gemm_nn_sub_x7
template <typename H>
__global__ __launch_bounds__(kThreads, 2) void gemm_half_sub_x7(int M, int N, int K, const H* __restrict__ Ah,
                                                                 int lda_h, const H* __restrict__ Bh, int ldb_h,
                                                                 const float* __restrict__ rs,
                                                                 const float* __restrict__ cs,
                                                                 float* __restrict__ C, int ldc, unsigned* ctr,
                                                                 unsigned* next) {
    const int nt = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
    claimed_tiles(ctr, next, nt, [&](int L) { gemm_half_tile<H>(L, M, N, K, Ah, lda_h, Bh, ldb_h, rs, cs, C, ldc); });
}

}  // namespace

// Grid of a launch that leaves XCD 0 free: two work-groups per CU (those
// dealt to XCD 0 return at once), no more than there are tiles plus one round.
inline int x7_grid(int num_cus, int tiles) { return std::min(2 * num_cus, tiles + tiles / 7 + 8); }

template <typename T>
int launch_gemm(int M, int N, int K, const T* A, int lda, const T* B, int ldb, T* C, int ldc,
                hipStream_t stream, XcdClaim claim) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    const int tiles = ((M + kLuBM - 1) / kLuBM) * ((N + kBN - 1) / kBN);
    if (claim.ctr)
        hipLaunchKernelGGL((gemm_nn_sub_x7<T, 16>), dim3(std::min(3 * claim.cus, tiles + tiles / 7 + 8)),
                           dim3(kThreads), 0, stream, M, N, K, A, lda, B, ldb, C, ldc, claim.ctr, claim.next);
    else
        hipLaunchKernelGGL((gemm_nn_sub<T, 16>), dim3(tiles), dim3(kThreads), 0, stream, M, N, K, A, lda, B,
                           ldb, C, ldc);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_gemm_hh(int M, int N, int K, const T* A, int lda, const T* B, int ldb, T* C, int ldc,
                   hipStream_t stream) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    const long long tiles = (long long)((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
    if (tiles > 0x7fffffffLL) return -1;
    hipLaunchKernelGGL((gemm_nn_hh<T, 16>), dim3((unsigned)tiles), dim3(kThreads), 0, stream, M, N, K, A, lda, B,
                       ldb, C, ldc);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T>
int launch_gemm_split(int M, int N, int K, int ks, const T* A, int lda, const T* B, int ldb, T* C, int ldc,
                      long long cstride, hipStream_t stream) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    if (ks <= 0) return -1;
    const int tiles = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
    const int splits = (K + ks - 1) / ks;
    if (splits > 65535) return -1;
    hipLaunchKernelGGL((gemm_nn_split<T, 16>), dim3(tiles, splits), dim3(kThreads), 0, stream, M, N, K, ks, A,
                       lda, B, ldb, C, ldc, cstride);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T>
int launch_syrk_lower(int M, int N, int K, const T* A, int lda, const T* B, int ldb, T* C, int ldc, int diag,
                      hipStream_t stream) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    const long long tiles = (long long)((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
    if (tiles > 0x7fffffffLL) return -1;
    hipLaunchKernelGGL((syrk_ln_sub<T, 16>), dim3((unsigned)tiles), dim3(kThreads), 0, stream, M, N, K, A, lda,
                       B, ldb, C, ldc, diag);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename H>
int launch_gemm_half(int M, int N, int K, const H* Ah, int lda_h, const H* Bh, int ldb_h,
                     const float* rs, const float* cs, float* C, int ldc, hipStream_t stream, XcdClaim claim) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    const int tiles = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
    if (claim.ctr)
        hipLaunchKernelGGL((gemm_half_sub_x7<H>), dim3(x7_grid(claim.cus, tiles)), dim3(kThreads), 0, stream, M, N, K,
                           Ah, lda_h, Bh, ldb_h, rs, cs, C, ldc, claim.ctr, claim.next);
    else
        hipLaunchKernelGGL((gemm_half_sub<H>), dim3(tiles), dim3(kThreads), 0, stream, M, N, K, Ah, lda_h, Bh,
                           ldb_h, rs, cs, C, ldc);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_gemm<double>(int, int, int, const double*, int, const double*, int, double*, int,
                                 hipStream_t, XcdClaim);
template int launch_gemm<float>(int, int, int, const float*, int, const float*, int, float*, int, hipStream_t, XcdClaim);
template int launch_gemm_hh<double>(int, int, int, const double*, int, const double*, int, double*, int,
                                    hipStream_t);
template int launch_gemm_split<double>(int, int, int, int, const double*, int, const double*, int, double*, int,
                                       long long, hipStream_t);
template int launch_syrk_lower<double>(int, int, int, const double*, int, const double*, int, double*, int, int,
                                       hipStream_t);
template int launch_gemm_half<_Float16>(int, int, int, const _Float16*, int, const _Float16*, int,
                                        const float*, const float*, float*, int, hipStream_t, XcdClaim);
template int launch_gemm_half<__bf16>(int, int, int, const __bf16*, int, const __bf16*, int, const float*,
                                      const float*, float*, int, hipStream_t, XcdClaim);

// One MFMA on lane-indexed values, to check the operand/result lane layout.
__global__ void probe_mfma_f64_kernel(double* out) {
    const int l = threadIdx.x;
    v4d c = {0, 0, 0, 0};
    c = __builtin_amdgcn_mfma_f64_16x16x4f64((double)l, 100.0 + l, c, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = c[r];
}

int launch_probe_mfma_f64(double* out, hipStream_t stream) {
    hipLaunchKernelGGL(probe_mfma_f64_kernel, dim3(1), dim3(64), 0, stream, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace lu
