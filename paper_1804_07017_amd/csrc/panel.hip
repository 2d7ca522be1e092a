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

constexpr int kPanelThreads = 256;
constexpr int kUChunk = 32;   // right-hand columns staged per pass of the in-panel update

template <typename T, int NB>
struct PanelShared {
    T red_v[4];
    int red_i[4];
    int win_i;
    int win_g;
    T prow[NB];
    T drow[NB];
    T L[NB][NB + 1];
    T U[NB][kUChunk];
    int piv[kMovesMaxW];          // panel-relative pivot rows of every column so far
    int bmv[1 + 4 * NB];          // block moves: count, (dst, src)...
    MovesScratch ms;
};

template <typename T, int NB, int RPT>
__global__ __launch_bounds__(kPanelThreads) void panel_kernel(PanelArgs<T> a) {
    __shared__ PanelShared<T, NB> sh;
    const int tid = threadIdx.x;
    const int g = blockIdx.x;
    const int P = gridDim.x;
    const int R = kPanelThreads * RPT;
    const int m = a.m, w = a.w;
    const long long lda = a.lda;
    T* __restrict__ A = a.A;
    unsigned epoch = 0;

    if (g == 0 && tid == 0 && a.sync_next) {
        a.sync_next[0] = 0u;   // counter of the next launch's slot (its previous user has finished)
    }

    auto row_of = [&](int q) { return g * R + q * kPanelThreads + tid; };

    T reg[RPT][NB];

    for (int cb = 0; cb < w; cb += NB) {
        const int nbw = (w - cb) < NB ? (w - cb) : NB;
        // load the block
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = row_of(q);
#pragma unroll
            for (int jj = 0; jj < NB; ++jj)
                reg[q][jj] = (i < m && jj < nbw) ? A[i + (long long)(cb + jj) * lda] : T(0);
        }

#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j < nbw) {
                const int d = cb + j;
                const int par = (epoch & 1u);
                // 1. local arg-max over rows >= d
                T bv = T(-1);
                int bi = 0x7fffffff;
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int i = row_of(q);
                    if (i >= d && i < m) argmax_merge(bv, bi, dabs(reg[q][j]), i);
                }
                wave_argmax(bv, bi);
                if ((tid & (kWave - 1)) == 0) { sh.red_v[tid / kWave] = bv; sh.red_i[tid / kWave] = bi; }
                __syncthreads();
                if (tid == 0) {
#pragma unroll
                    for (int wv = 1; wv < kPanelThreads / kWave; ++wv) argmax_merge(bv, bi, sh.red_v[wv], sh.red_i[wv]);
                    sh.win_i = bi;
                    a.cand_val[par * P + g] = bv;
                    a.cand_idx[par * P + g] = bi;
                }
                __syncthreads();
                // 2. publish the local winner's row and, from its owner, row d
                {
                    const int wi = sh.win_i;
#pragma unroll
                    for (int q = 0; q < RPT; ++q) {
                        const int i = row_of(q);
                        if (i == wi) {
#pragma unroll
                            for (int jj = 0; jj < NB; ++jj) a.cand_rows[(par * P + g) * NB + jj] = reg[q][jj];
                        }
                        if (i == d) {
#pragma unroll
                            for (int jj = 0; jj < NB; ++jj) a.diag_rows[par * NB + jj] = reg[q][jj];
                        }
                    }
                }
                if (grid_barrier(a.sync, a.sync + 1, ++epoch, a.spin_limit)) return;
                // 3. global winner (same decision in every work-group)
                if (tid < kWave) {
                    T v = T(-1);
                    int i = 0x7fffffff, gg = 0x7fffffff;
                    for (int c = tid; c < P; c += kWave) {
                        T cv = a.cand_val[par * P + c];
                        int ci = a.cand_idx[par * P + c];
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
                    sh.drow[tid] = a.diag_rows[par * NB + tid];
                    sh.prow[tid] = (wg >= 0) ? a.cand_rows[(par * P + wg) * NB + tid] : a.diag_rows[par * NB + tid];
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
                // 4. interchange rows d and p inside the block, scale, rank-1 update
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int i = row_of(q);
                    if (p != d) {
                        if (i == p) {
#pragma unroll
                            for (int jj = 0; jj < NB; ++jj) reg[q][jj] = sh.drow[jj];
                        } else if (i == d) {
#pragma unroll
                            for (int jj = 0; jj < NB; ++jj) reg[q][jj] = sh.prow[jj];
                        }
                    }
                    if (i > d && i < m) {
                        T l = reg[q][j];
                        if (piv != T(0)) l = l / piv;
                        reg[q][j] = l;
#pragma unroll
                        for (int jj = j + 1; jj < NB; ++jj) reg[q][jj] = reg[q][jj] - l * sh.prow[jj];
                    }
                }
            }
        }

        // write the factored block back
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = row_of(q);
            if (i < m) {
#pragma unroll
                for (int jj = 0; jj < NB; ++jj)
                    if (jj < nbw) A[i + (long long)(cb + jj) * lda] = reg[q][jj];
            }
        }

        const bool more_cols = (w - cb - nbw) > 0 || cb > 0;
        if (more_cols) {
            const int gd = cb / R;     // owner of the block's diagonal rows
            if (g == gd) {
                // block L11 (unit lower) into LDS, from the owners' registers
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int r = row_of(q) - cb;
                    if (r >= 0 && r < nbw) {
#pragma unroll
                        for (int jj = 0; jj < NB; ++jj) sh.L[r][jj] = reg[q][jj];
                    }
                }
                if (tid == 0) {
                    // compose the block's nbw interchanges (tiny: sequential)
                    int slot_row[2 * NB], content[2 * NB];
                    int ns = nbw;
                    for (int s = 0; s < nbw; ++s) { slot_row[s] = cb + s; content[s] = cb + s; }
                    for (int s = 0; s < nbw; ++s) {
                        const int pr = sh.piv[cb + s];
                        int sb;
                        if (pr < cb + nbw) {
                            sb = pr - cb;
                        } else {
                            sb = -1;
                            for (int e = nbw; e < ns; ++e) if (slot_row[e] == pr) { sb = e; break; }
                            if (sb < 0) { sb = ns++; slot_row[sb] = pr; content[sb] = pr; }
                        }
                        int tmp = content[s]; content[s] = content[sb]; content[sb] = tmp;
                    }
                    int cnt = 0;
                    for (int s = 0; s < ns; ++s)
                        if (content[s] != slot_row[s]) { sh.bmv[1 + 2 * cnt] = slot_row[s]; sh.bmv[2 + 2 * cnt] = content[s]; ++cnt; }
                    sh.bmv[0] = cnt;
                }
                __syncthreads();
                const int cnt = sh.bmv[0];
                // interchanges on the other panel columns; TRSM on the right ones
                for (int c = tid; c < w - nbw; c += kPanelThreads) {
                    const int col = (c < cb) ? c : c + nbw;
                    T* colp = A + (long long)col * lda;
                    T v[2 * NB];
#pragma unroll
                    for (int s = 0; s < 2 * NB; ++s)
                        if (s < cnt) v[s] = colp[sh.bmv[2 + 2 * s]];
#pragma unroll
                    for (int s = 0; s < 2 * NB; ++s)
                        if (s < cnt) colp[sh.bmv[1 + 2 * s]] = v[s];
                    if (col >= cb + nbw) {
                        T x[NB];
#pragma unroll
                        for (int r = 0; r < NB; ++r) x[r] = (r < nbw) ? colp[cb + r] : T(0);
#pragma unroll
                        for (int s = 0; s < NB; ++s) {
#pragma unroll
                            for (int r = s + 1; r < NB; ++r) x[r] = x[r] - sh.L[r][s] * x[s];
                        }
#pragma unroll
                        for (int r = 0; r < NB; ++r)
                            if (r < nbw) colp[cb + r] = x[r];
                    }
                }
            }
            if (grid_barrier(a.sync, a.sync + 1, ++epoch, a.spin_limit)) return;
            // in-panel trailing update of my rows below the block: A[i, right] -= L[i, blk] U[blk, right]
            const int right0 = cb + nbw;
            for (int c0 = right0; c0 < w; c0 += kUChunk) {
                const int nc = (w - c0) < kUChunk ? (w - c0) : kUChunk;
                for (int e = tid; e < NB * kUChunk; e += kPanelThreads) {
                    const int s = e % NB, cc = e / NB;
                    sh.U[s][cc] = (s < nbw && cc < nc) ? A[(cb + s) + (long long)(c0 + cc) * lda] : T(0);
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int i = row_of(q);
                    if (i >= right0 && i < m) {
                        T l[NB];   // this row's block of L, re-read (the registers were released)
#pragma unroll
                        for (int s = 0; s < NB; ++s) l[s] = (s < nbw) ? A[i + (long long)(cb + s) * lda] : T(0);
                        for (int cc = 0; cc < nc; ++cc) {
                            T* p = A + i + (long long)(c0 + cc) * lda;
                            T x = *p;
#pragma unroll
                            for (int s = 0; s < NB; ++s) x = x - l[s] * sh.U[s][cc];
                            *p = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }

    // compose the whole panel's interchanges for the trailing kernels
    if (g == 0 && a.moves) {
        __syncthreads();
        compose_moves(sh.piv, w, a.moves, sh.ms);
    }
    (void)P;
}

}  // namespace

template <typename T>
int launch_panel(const PanelArgs<T>& args, int wgs, hipStream_t stream) {
    // NB = 16 for both precisions; rows per thread chosen so that wgs * 256 * RPT >= m.
    constexpr int NB = 16;
    const int m = args.m;
    int rpt = (m + wgs * kPanelThreads - 1) / (wgs * kPanelThreads);
    if (rpt < 1) rpt = 1;
    dim3 block(kPanelThreads);
    if (rpt == 1) {
        hipLaunchKernelGGL((panel_kernel<T, NB, 1>), dim3(wgs), block, 0, stream, args);
    } else if (rpt == 2) {
        hipLaunchKernelGGL((panel_kernel<T, NB, 2>), dim3(wgs), block, 0, stream, args);
    } else if (rpt <= 4) {
        hipLaunchKernelGGL((panel_kernel<T, NB, 4>), dim3(wgs), block, 0, stream, args);
    } else {
        return -1;   // caller must raise wgs
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int panel_max_rows_per_wg() { return kPanelThreads * 4; }

template int launch_panel<double>(const PanelArgs<double>&, int, hipStream_t);
template int launch_panel<float>(const PanelArgs<float>&, int, hipStream_t);

}  // namespace lu
