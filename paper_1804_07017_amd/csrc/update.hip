// Row interchanges and the U12 triangular solve of one elimination step
// (paper Sec. 3.4: laswp and trsm of getrf; Sec. 3.5: RL2 of LU_blk,
// A12 := trilu(A11)^-1 A12, trilu = the unit lower triangle).
//
// swap_trsm_kernel: LASWP and RL2 (A12 := trilu(A11)^-1 A12, paper Sec. 3.5)
// for one slab of BN columns per work-group:
//   1. gather: the w top rows of the slab, with the panel's composed
//      interchanges applied, straight into matrix-core accumulators; then the
//      rows displaced below the top w rows are written out (every read of the
//      slab is done by then);
//   2. blocked forward substitution with 16-row blocks: block row i is
//      finished as X_i = inv(L_ii) X_i (the 16x16 unit-lower inverses come from
//      diag_inv_kernel), then every block row below takes X_j -= L_ji X_i --
//      both on the FP64/FP32 matrix cores, X staying in registers;
//   3. U12 goes back to the matrix (and, in the mixed-precision mode, to a
//      half-precision copy with one power-of-two scale per column).
// lswap_kernel: the same interchanges on finished columns left of the panel.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"
#include "moves.hpp"

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

// Inverses of the 16x16 unit-lower diagonal blocks of L11 (w x w at (r0, r0)):
// linv[blk*256 + k*16 + j] = inv(L_blk)[j][k] (column-major blocks); rows and
// columns past w are taken from the identity.  One 64-thread work-group per
// block; lane j < 16 solves for column j.
template <typename T>
__global__ __launch_bounds__(64) void diag_inv_kernel(const T* __restrict__ A, long long lda, int r0, int w,
                                                      T* __restrict__ linv) {
    __shared__ T Lb[16][17];
    __shared__ T Y[16][17];
    const int blk = blockIdx.x, l = threadIdx.x;
    const int b0 = blk * 16;
    for (int e = l; e < 256; e += 64) {
        const int i = e % 16, k = e / 16;
        const bool in = b0 + i < w && b0 + k < w && i > k;
        Lb[i][k] = in ? A[(r0 + b0 + i) + (long long)(r0 + b0 + k) * lda] : T(0);
    }
    __syncthreads();
    if (l < 16) {
        const int j = l;
        for (int r = 0; r < 16; ++r) Y[r][j] = (r == j) ? T(1) : T(0);
        for (int r = j + 1; r < 16; ++r) {
            T acc = T(0);
            for (int q = j; q < r; ++q) acc += Lb[r][q] * Y[q][j];
            Y[r][j] = -acc;
        }
    }
    __syncthreads();
    for (int e = l; e < 256; e += 64) {
        const int j = e % 16, k = e / 16;           // inv[j][k] at k*16 + j
        linv[(size_t)blk * 256 + e] = Y[j][k];
    }
}

// ROWT row tiles (16 rows each) per wave, NCT column tiles (16 columns) per
// work-group; wave v owns row tiles v, v+4, v+8, ...
template <typename T, typename H, int ROWT, int NCT>
__device__ __forceinline__ void swap_trsm_slab(const SwapTrsmArgs<T, H>& a, int slab) {
    typedef typename Acc<T>::type V4;
    constexpr int BN = 16 * NCT;
    constexpr int LDX = BN + 1;
    __shared__ int top_src[kMovesMaxW];
    __shared__ int ex_dst[kMovesMaxW];
    __shared__ int ex_src[kMovesMaxW];
    __shared__ T Xi[2][16][LDX];       // finished block row i (double-buffered)
    __shared__ T Ys[16][LDX];          // owner's staging of block row i before inv(L_ii)
    __shared__ unsigned colmax[BN];
    __shared__ int ex_count;

    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int l16 = lane % 16, lg = lane / 16;
    const int w = a.w;
    const int nrt = (w + 15) / 16;
    const int c_base = a.c0 + slab * BN;
    if (c_base >= a.c1) return;
    const long long lda = a.lda;
    T* __restrict__ Atop = a.A + a.r0;                  // row r0 of column 0
    const T* __restrict__ L = a.A + a.r0 + (long long)a.r0 * lda;   // L11 at (r0, r0)

    // the list is read defensively (moves.hpp): counts clamped, moves outside
    // the block dropped
    const int ntop = moves_top_count(a.moves, w);
    int nex = 0;
    const int mrows = a.m;
    for (int t = tid; t < w; t += kThreads) top_src[t] = t;
    if (tid == 0) ex_count = 0;
    __syncthreads();
    for (int s = tid; s < ntop; s += kThreads) {
        int dst, src;
        if (moves_top(a.moves, s, w, mrows, dst, src)) top_src[dst] = src;
    }
    for (int s = tid; s < moves_extra_count(a.moves, w); s += kThreads) {
        int dst, src;
        if (moves_extra(a.moves, s, w, mrows, dst, src)) {
            const int slot = atomicAdd(&ex_count, 1);
            ex_dst[slot] = dst;
            ex_src[slot] = src;
        }
    }
    if (tid < BN) colmax[tid] = 0u;
    __syncthreads();
    nex = ex_count;

    // 1. gather into the accumulators: lane (l16, lg), register r of tile
    //    (q, ct) holds X[row = (wave + 4q)*16 + l16][col = ct*16 + Acc::col(lg, r)]
    V4 acc[ROWT][NCT];
#pragma unroll
    for (int q = 0; q < ROWT; ++q) {
        const int t = (wave + 4 * q) * 16 + l16;
        const bool rok = t < w;
        const int src = rok ? top_src[t] : 0;
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int col = c_base + ct * 16 + Acc<T>::col(lg, r);
                const bool ok = rok && col < a.c1;
                const T v = Atop[src + (long long)(ok ? col : a.c0) * lda];
                acc[q][ct][r] = ok ? v : T(0);
            }
        }
    }
    __syncthreads();   // every read of the slab's moved rows is done
    // displaced top rows -> their rows below the top block (sources are
    // original top rows, not written before step 3)
    {
        constexpr int kB = 8;
        for (int e0 = tid; e0 < nex * BN; e0 += kThreads * kB) {
            T v[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int e = e0 + u * kThreads;
                const int s = e % max(nex, 1), c = c_base + e / max(nex, 1);
                const bool ok = e < nex * BN && c < a.c1;
                v[u] = Atop[(ok ? ex_src[s] : 0) + (long long)(ok ? c : a.c0) * lda];
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int e = e0 + u * kThreads;
                const int s = e % max(nex, 1), c = c_base + e / max(nex, 1);
                if (e < nex * BN && c < a.c1) Atop[ex_dst[s] + (long long)c * lda] = v[u];
            }
        }
    }

    // 2. blocked substitution; the L operand of the next step is prefetched
    //    into registers while the current step runs.
    //    lane l supplies L[row = rt*16 + l16][k = 16 i + 4 kk + lg]
    auto load_l = [&](int i, T (&dst)[ROWT][4]) {
#pragma unroll
        for (int q = 0; q < ROWT; ++q) {
            const int row = (wave + 4 * q) * 16 + l16;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 16 * i + 4 * kk + lg;
                const bool ok = row < w && k < w && (wave + 4 * q) > i;
                const T v = L[(ok ? row : 0) + (long long)(ok ? k : 0) * lda];
                dst[q][kk] = ok ? v : T(0);
            }
        }
    };
    // The owner of block row i+1 updates it with X_i and finishes it first
    // (the next step's critical path), then every wave updates its other rows.
    auto load_inv = [&](int i, T (&dst)[4]) {
        const T* __restrict__ inv = a.linv + (size_t)min(i, nrt - 1) * 256;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) dst[kk] = inv[(4 * kk + lg) * 16 + l16];   // B[k][j] = inv[j][k]
    };
    // finish block row i held in acc[i/4] of the calling wave: X_i = inv(L_ii) X_i
    auto finish = [&](int i, const T (&bi)[4]) {
        const int qi = i >> 2;
        const int buf = i & 1;
#pragma unroll
        for (int q = 0; q < ROWT; ++q) {
            if (q == qi) {
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
                    for (int r = 0; r < 4; ++r) Ys[l16][ct * 16 + Acc<T>::col(lg, r)] = acc[q][ct][r];
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);      // lgkmcnt(0): the wave's LDS writes are done
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            V4 d = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) d = mfma(Ys[4 * kk + lg][ct * 16 + l16], bi[kk], d);
#pragma unroll
            for (int r = 0; r < 4; ++r) Xi[buf][l16][ct * 16 + Acc<T>::col(lg, r)] = d[r];
#pragma unroll
            for (int q = 0; q < ROWT; ++q)
                if (q == qi) acc[q][ct] = d;
        }
    };
    auto update = [&](int q, int buf, const T (&l)[4]) {
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                acc[q][ct] = mfma(-Xi[buf][4 * kk + lg][ct * 16 + l16], l[kk], acc[q][ct]);
    };
    T lc[ROWT][4], ln[ROWT][4];
    T ic[4], in_[4];
    load_l(0, lc);
    load_inv(0, ic);
    if (wave == 0) finish(0, ic);
    load_inv(1, ic);
    __syncthreads();
    for (int i = 0; i < nrt; ++i) {
        const int buf = i & 1;
        if (i + 1 < nrt) load_l(i + 1, ln);
        if (i + 2 < nrt) load_inv(i + 2, in_);
        const int nxt = i + 1;
        const bool owner = nxt < nrt && wave == (nxt & 3);
        if (owner) {
#pragma unroll
            for (int q = 0; q < ROWT; ++q)
                if (q == (nxt >> 2)) update(q, buf, lc[q]);
            finish(nxt, ic);
        }
#pragma unroll
        for (int q = 0; q < ROWT; ++q) {
            const int rt = wave + 4 * q;
            if (rt > i && rt < nrt && !(owner && q == (nxt >> 2))) update(q, buf, lc[q]);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < ROWT; ++q)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) lc[q][kk] = ln[q][kk];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) ic[kk] = in_[kk];
    }

    // 3. U12 back to the matrix
#pragma unroll
    for (int q = 0; q < ROWT; ++q) {
        const int t = (wave + 4 * q) * 16 + l16;
        if (t < w) {
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int col = c_base + ct * 16 + Acc<T>::col(lg, r);
                    if (col < a.c1) Atop[t + (long long)col * lda] = acc[q][ct][r];
                }
        }
    }
    if (a.uh) {
        // per-column amax over the w rows -> power-of-two scale -> half copy
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float m = 0.f;
#pragma unroll
                for (int q = 0; q < ROWT; ++q)
                    if ((wave + 4 * q) * 16 + l16 < w) m = fmaxf(m, fabsf((float)acc[q][ct][r]));
#pragma unroll
                for (int off = 8; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
                if (l16 == 0) atomicMax(&colmax[ct * 16 + Acc<T>::col(lg, r)], __float_as_uint(m));
            }
        __syncthreads();
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int cc = ct * 16 + Acc<T>::col(lg, r);
                const int col = c_base + cc;
                if (col >= a.c1) continue;
                const float sc = pow2_scale(__uint_as_float(colmax[cc]));
                if (wave == 0 && l16 == 0) a.cs[col] = 1.f / sc;
#pragma unroll
                for (int q = 0; q < ROWT; ++q) {
                    const int t = (wave + 4 * q) * 16 + l16;
                    if (t < w) a.uh[(long long)col * a.lduh + t] = (H)((float)acc[q][ct][r] * sc);
                }
            }
    }
}

// One slab per work-group, or -- beside a panel that holds XCD 0 -- the
// work-groups on XCD 0 return at once and the others claim slabs from a
// counter until none is left (a counter of the launch before, which has
// finished on this stream, is cleared here for the next launch).
template <typename T, typename H, int ROWT, int NCT>
__global__ __launch_bounds__(kThreads, 2) void swap_trsm_kernel(SwapTrsmArgs<T, H> a) {
    constexpr int BN = 16 * NCT;
    if (!a.claim) {
        swap_trsm_slab<T, H, ROWT, NCT>(a, blockIdx.x);
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) xstore(a.claim_next, 0u);
    if (xcd_id() == 0) return;
    const int nslabs = (a.c1 - a.c0 + BN - 1) / BN;
    __shared__ int s_slab;
    for (;;) {
        __syncthreads();                 // the previous slab's shared-memory reads are done
        if (threadIdx.x == 0) s_slab = (int)atomicAdd(a.claim, 1u);
        __syncthreads();
        const int slab = s_slab;
        if (slab >= nslabs) break;
        swap_trsm_slab<T, H, ROWT, NCT>(a, slab);
    }
}

// Interchanges only, on columns [c0, c1): all reads of a column before its writes.
// The list is read as in swap_trsm_kernel (rows relative to r0, m rows from there).
template <typename T>
__global__ __launch_bounds__(kThreads) void lswap_kernel(T* A, long long lda, int r0, int w, int m, const int* moves,
                                                         int c0, int c1, int cols_per_wg, unsigned* claim,
                                                         unsigned* claim_next) {
    __shared__ int mv[2 * 2 * kMovesMaxW];   // (dst, src) pairs, top then extra
    const int tid = threadIdx.x;
    if (claim && blockIdx.x == 0 && threadIdx.x == 0) xstore(claim_next, 0u);
    if (claim && xcd_id() == 0) return;      // XCD 0 is left to the panel
    __shared__ int cnt_s;
    if (tid == 0) cnt_s = 0;
    __syncthreads();
    // the list is read defensively (moves.hpp): moves outside the block are dropped
    for (int s = tid; s < moves_top_count(moves, w); s += kThreads) {
        int dst, src;
        if (moves_top(moves, s, w, m, dst, src)) {
            const int slot = atomicAdd(&cnt_s, 1);
            mv[2 * slot] = dst;
            mv[2 * slot + 1] = src;
        }
    }
    for (int s = tid; s < moves_extra_count(moves, w); s += kThreads) {
        int dst, src;
        if (moves_extra(moves, s, w, m, dst, src)) {
            const int slot = atomicAdd(&cnt_s, 1);
            mv[2 * slot] = dst;
            mv[2 * slot + 1] = src;
        }
    }
    __syncthreads();
    const int cnt = cnt_s;
    constexpr int kPer = (2 * kMovesMaxW + kThreads - 1) / kThreads;
    __shared__ int s_blk;
    const int nblk = (c1 - c0 + cols_per_wg - 1) / cols_per_wg;
    for (int it = 0;; ++it) {
      int blk;
      if (claim) {                              // blocks of columns claimed from a counter
          __syncthreads();
          if (tid == 0) s_blk = (int)atomicAdd(claim, 1u);
          __syncthreads();
          blk = s_blk;
      } else {
          blk = it == 0 ? (int)blockIdx.x : nblk;
      }
      if (blk >= nblk) break;
      const int cb = c0 + blk * cols_per_wg;
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
}

// Left interchanges deferred to the end of the factorization (the LPERM task):
// the columns of panel k take the interchanges of every later panel j > k, on
// rows >= r0 = starts[k+1], as one permutation sigma_k of those rows, where
// applying panels k+1, k+2, ... in order to a column gives new[r] =
// old[sigma_k(r)].  With M_j the permutation of panel j's composed moves
// (new[dst] = old[src]), sigma_k = M_{k+1} o sigma_{k+1} and so
// sigma_k^-1 = sigma_{k+1}^-1 o M_{k+1}^-1: starting from the identity and
// taking the panels from the last one down to k+1, each panel's moves set
// inv[src] = inv[dst] (all reads before the writes).  Then every column
// segment is read whole into registers and written back permuted,
// new[inv[i]] = old[i].  Work-group b takes kLpermCols columns of one panel
// (panels in order, ceil(w_k / kLpermCols) work-groups each) and rebuilds
// that panel's inv in LDS.  The moves are read defensively (moves.hpp).
template <typename T>
__global__ __launch_bounds__(kLpermThreads) void lperm_kernel(T* A, long long lda, int n, int N,
                                                             const int* __restrict__ starts,
                                                             const int* __restrict__ moves) {
    extern __shared__ int inv[];
    const int tid = threadIdx.x;
    int b = blockIdx.x, k = 0;
    for (; k < N - 1; ++k) {
        const int nb = (starts[k + 1] - starts[k] + kLpermCols - 1) / kLpermCols;
        if (b < nb) break;
        b -= nb;
    }
    if (k >= N - 1) return;
    const int r0 = starts[k + 1], L = n - r0;
    const int c0 = starts[k] + b * kLpermCols, c1 = min(starts[k + 1], c0 + kLpermCols);
    for (int i = tid; i < L; i += kLpermThreads) inv[i] = i;
    __syncthreads();
    for (int j = N - 1; j > k; --j) {
        const int* mv = moves + (size_t)j * kMovesLen;
        const int wj = starts[j + 1] - starts[j], mj = n - starts[j], o = starts[j] - r0;
        const int nt = moves_top_count(mv, wj), ne = moves_extra_count(mv, wj);
        int d = -1, src = 0, val = 0;
        if (tid < nt) {
            int dd, ss;
            if (moves_top(mv, tid, wj, mj, dd, ss)) { d = dd + o; src = ss + o; }
        } else if (tid < nt + ne) {
            int dd, ss;
            if (moves_extra(mv, tid - nt, wj, mj, dd, ss)) { d = dd + o; src = ss + o; }
        }
        if (d >= 0) val = inv[d];
        __syncthreads();
        if (d >= 0) inv[src] = val;
        __syncthreads();
    }
    constexpr int V = kLpermMaxRows / kLpermThreads;
    for (int c = c0; c < c1; ++c) {
        T* col = A + r0 + (long long)c * lda;
        T v[V];
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const int i = tid + u * kLpermThreads;
            if (i < L) v[u] = col[i];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const int i = tid + u * kLpermThreads;
            if (i < L) col[inv[i]] = v[u];
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
int launch_swap_trsm(const SwapTrsmArgs<T, H>& args, hipStream_t stream) {
    if (args.c1 <= args.c0 || args.w <= 0) return 0;
    if (args.w > kMovesMaxW || !args.linv) return -1;
    const int nrt = (args.w + 15) / 16;
    const int ncols = args.c1 - args.c0;
    auto go = [&](auto kern, int bn) {
        const int slabs = (ncols + bn - 1) / bn;
        // claimed slabs: about as many work-groups as slabs, at most two per CU
        const int grid = args.claim ? std::min(slabs + slabs / 7 + 8, 512) : slabs;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, stream, args);
    };
    if (nrt <= 4) go(swap_trsm_kernel<T, H, 1, 4>, 64);
    else if (nrt <= 8) go(swap_trsm_kernel<T, H, 2, 4>, 64);
    else if constexpr (sizeof(T) == 4) {  // FP32 accumulators are half the size: wider slabs
        if (nrt <= 16) go(swap_trsm_kernel<T, H, 4, 4>, 64);
        else go(swap_trsm_kernel<T, H, 8, 2>, 32);
    } else {
        if (nrt <= 16) go(swap_trsm_kernel<T, H, 4, 2>, 32);
        else go(swap_trsm_kernel<T, H, 8, 1>, 16);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_diag_inv(const T* A, long long lda, int r0, int w, T* linv, hipStream_t stream) {
    if (w <= 0) return 0;
    hipLaunchKernelGGL((diag_inv_kernel<T>), dim3((w + 15) / 16), dim3(64), 0, stream, A, lda, r0, w, linv);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_diag_inv<double>(const double*, long long, int, int, double*, hipStream_t);
template int launch_diag_inv<float>(const float*, long long, int, int, float*, hipStream_t);

template <typename T>
int launch_lswap(T* A, long long lda, int r0, int w, int m, const int* moves, int c0, int c1, hipStream_t stream,
                 unsigned* claim, unsigned* claim_next) {
    if (c1 <= c0 || m <= 0) return 0;
    if (w < 1 || w > kMovesMaxW) return -1;
    const int per = 4;
    const int blocks = (c1 - c0 + per - 1) / per;
    const int grid = claim ? std::min(blocks + blocks / 7 + 8, 1024) : blocks;
    hipLaunchKernelGGL((lswap_kernel<T>), dim3(grid), dim3(kThreads), 0, stream, A, lda, r0, w, m, moves, c0, c1,
                       per, claim, claim_next);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_lperm(T* A, long long lda, int n, int N, const int* starts_host, const int* starts_dev, const int* moves,
                 hipStream_t stream) {
    if (N < 2) return 0;
    if (n - starts_host[1] > kLpermMaxRows) return -1;
    int wgs = 0;
    for (int k = 0; k + 1 < N; ++k) wgs += (starts_host[k + 1] - starts_host[k] + kLpermCols - 1) / kLpermCols;
    const size_t lds = sizeof(int) * (size_t)(n - starts_host[1]);
    static bool attr_set = false;           // dynamic LDS beyond the default limit
    if (!attr_set) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&lperm_kernel<T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(sizeof(int) * kLpermMaxRows)) != hipSuccess)
            return -1;
        attr_set = true;
    }
    hipLaunchKernelGGL((lperm_kernel<T>), dim3(wgs), dim3(kLpermThreads), lds, stream, A, lda, n, N, starts_dev,
                       moves);
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
template int launch_lperm<double>(double*, long long, int, int, const int*, const int*, const int*, hipStream_t);
template int launch_lperm<float>(float*, long long, int, int, const int*, const int*, const int*, hipStream_t);
template int launch_lswap<double>(double*, long long, int, int, int, const int*, int, int, hipStream_t, unsigned*,
                                  unsigned*);
template int launch_lswap<float>(float*, long long, int, int, int, const int*, int, int, hipStream_t, unsigned*,
                                 unsigned*);
template int launch_l21_half<_Float16>(const float*, long long, int, int, _Float16*, long long, float*,
                                       hipStream_t);
template int launch_l21_half<__bf16>(const float*, long long, int, int, __bf16*, long long, float*, hipStream_t);

}  // namespace lu
