// Householder QR with look-ahead: A = Q R, Q = H_0 H_1 ... with
// H_j = I - tau_j v_j v_j^T (LAPACK geqrf storage: R on and above the
// diagonal, v below it with v_j = 1 implicit).  QR fits the blocked skeleton
// of the paper (Sec. 3.1): per iteration the panel is factored with
// Householder reflectors and their block form Q_k = I - V T V^T (T upper
// triangular) is applied to the trailing matrix, C <- Q_k^T C =
// C - V (T^T (V^T C)); the look-ahead of Sec. 4 applies unchanged.
//
// Panel kernel: one persistent launch of P = ceil(m / 1024) work-groups (256
// threads each), group g owning the 1024-row block starting at g*1024 and
// thread t its rows g*1024 + t + s*256 (s < 4).  The panel is processed in
// inner blocks of 16 columns that each thread holds in registers for its rows,
// as a ring of 16 slots with the current column in slot 0.
// Per column J of an inner block, with two device-wide barriers (without
// cache maintenance: the few words exchanged use device-scope atomics):
//   1. each group's partial sum of squares below the diagonal (the owner of
//      row J also publishes the diagonal entry) -> barrier;
//   2. every group forms the same reflector (beta, tau, 1/(alpha - beta)) from
//      the partials summed in group order and scales its rows of v;
//   3. each group's partial dot products of v with the other columns of the
//      inner block (rows >= J) -> barrier;
//   4. every group sums them in group order, applies the reflector to its rows
//      of the inner block's columns right of J and extends the inner block's
//      T (T_b[0:j, j] = -tau_J T_b[0:j, 0:j] (V_b[:, 0:j]^T v_J), T_b[j, j] = tau_J).
// After an inner block (V_b, T_b), with two more barriers: each group's partial
// W = V_b^T A[:, c] over its rows for every panel column c outside the block
// -> barrier; the P partials summed in group order, spread over all groups ->
// barrier; then every group applies A[:, c] -= V_b (T_b^T W[:, c]) to its rows
// of the columns right of the block, and the columns left of it (their
// V^T V_b) give T's block above T_b: T[0:cb, b] = -T[0:cb, 0:cb] (V^T V_b) T_b.
// The per-column steps touch no memory; the panel is read and written once per
// inner block.  P and the rows of each group follow from m alone, and every
// sum runs in a fixed order (rows s, lanes by butterfly, waves, then groups),
// so the factorization of a given panel is bitwise the same whatever the
// schedule.
#include "common.hpp"
#include "kernels.hpp"

namespace lu {

namespace {

constexpr int kQrThreads = 256;
constexpr int kQrRows = kQrPanelGroupRows / 256;   // panel rows per thread
constexpr int kQrGroupRows = kQrThreads * kQrRows;
constexpr int kQrMaxW = kQrMaxPanelW;   // the widest panel: QR block size, band width
constexpr int kQrNB = 16;           // columns of an inner block (held in registers)
constexpr int kQrWaves = kQrThreads / kWave;
constexpr int kQrWc = 2;                         // columns per chunk of the block phase
constexpr int kQrWv = kQrWc * kQrNB;             // values per lane per chunk
constexpr int kQrRound = 512 / kQrWv;            // chunks per LDS round
// partial-sum workspace (doubles)
constexpr int kQrMaxGroups = kQrPanelMaxGroups;
constexpr int kPartSs = 0;                                            // [groups] sums of squares
constexpr int kPartAlpha = kQrMaxGroups;                              // the diagonal entry of column J
constexpr int kPartDot = 2 * kQrMaxGroups;                            // [groups][16] in-block dot products
constexpr int kPartW = kPartDot + kQrMaxGroups * kQrNB;               // [groups][16 * w] partial W
constexpr int kPartWs = kPartW + kQrMaxGroups * kQrNB * kQrMaxW;      // [16 * w] summed W
static_assert(kPartWs + kQrNB * kQrMaxW == kQrPartWords, "QR workspace layout");

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum over the 64 lanes of a[0..N-1] (N a power of two <= 64) by a butterfly
// that halves the vector at each exchange: on return the total of element
// lane / (64 / N) is in a[0].  The order of the additions is fixed.
template <int N>
__device__ __forceinline__ double wave_reduce_scatter(double (&a)[N], int lane) {
    int mask = 32;
#pragma unroll
    for (int half = N / 2; half >= 1; half >>= 1, mask >>= 1) {
        const bool up = (lane & mask) != 0;
#pragma unroll
        for (int k = 0; k < half; ++k) {
            const double lo = a[k], hi = a[k + half];
            const double send = up ? lo : hi;
            const double keep = up ? hi : lo;
            a[k] = keep + __shfl_xor(send, mask, kWave);
        }
    }
#pragma unroll
    for (; mask >= 1; mask >>= 1) a[0] = a[0] + __shfl_xor(a[0], mask, kWave);
    return a[0];
}

struct QrShared {
    double red[kQrWaves][kQrRound][kQrWv];  // block phase: wave totals of a round of chunks
    double rw[kQrWaves][kQrNB];             // column step: wave totals
    double dsum[kQrNB];                     // column step: summed dot products
    double Tb[kQrNB][kQrNB];                // T of the inner block (upper)
    double Ys[kQrNB][kQrMaxW];              // T_b^T W of the columns right of the block
    double Us[kQrMaxW][kQrNB];              // (V^T V_b) T_b of the columns left of it
    double sc[4];                           // tau, scal, beta
    double pss[kQrMaxGroups + 1];           // the groups' sums of squares, then the diagonal entry
    double pdot[kQrMaxGroups * kQrNB];      // the groups' dot products
};

// Where a thread is: its group, lanes and first row.
struct QrPos {
    int tid, lane, wave, g, P, row0;
};

// The per-column exchange words (partial sums, the diagonal entry) are read
// and written with device-scope atomics, which bypass the per-XCD L2, so the
// two barriers of a column need no cache write-back or invalidation.
__device__ __forceinline__ void st_dev(double* p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double* p) {
    return __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// One slot of the inner block's register ring forward: slot p takes slot p+1's
// column, slot 15 the column of slot 0.
__device__ __forceinline__ void qr_rotate(double (&X)[kQrRows][kQrNB]) {
#pragma unroll
    for (int s = 0; s < kQrRows; ++s) {
        const double t = X[s][0];
#pragma unroll
        for (int q = 0; q + 1 < kQrNB; ++q) X[s][q] = X[s][q + 1];
        X[s][kQrNB - 1] = t;
    }
}

// Column J = cb + jj of the inner block (steps 1-4 of the header); false when
// a barrier timed out.  The block is a ring of 16 register slots: on entry
// slot 0 holds column J, slot p (p < 16 - jj) column J + p and slot 16 - jj + l
// the finished column cb + l (l < jj); on return the ring has moved one slot
// forward.  One copy of this code serves every column (static slot indices).
__device__ __forceinline__ bool qr_column(double (&X)[kQrRows][kQrNB], QrShared& sh, const QrPanelArgs& a,
                                          const QrPos& p, int cb, int nbw, int jj, unsigned& epoch) {
    const int tid = p.tid, lane = p.lane, wave = p.wave, g = p.g, P = p.P, row0 = p.row0;
    const int m = a.m;
    double* part = a.part;
    const int J = cb + jj;
    // 1. partial sum of squares below the diagonal; the owner of row J
    //    publishes the diagonal entry
    double ss = 0.0;
#pragma unroll
    for (int s = 0; s < kQrRows; ++s) {
        const int i = row0 + s * kQrThreads;
        if (i > J && i < m) ss = ss + X[s][0] * X[s][0];
        if (i == J) st_dev(&part[kPartAlpha], X[s][0]);
    }
    ss = wave_sum(ss);
    if (lane == 0) sh.rw[wave][0] = ss;
    __syncthreads();
    if (tid == 0) st_dev(&part[kPartSs + g], (sh.rw[0][0] + sh.rw[1][0]) + (sh.rw[2][0] + sh.rw[3][0]));
    if (grid_barrier(a.sync, a.sync + 1, ++epoch, a.spin_limit, false)) return false;
    // 2. the reflector, identical in every group (the partials loaded in
    //    parallel, summed in group order)
    if (tid < P) sh.pss[tid] = ld_dev(&part[kPartSs + tid]);
    if (tid == kQrThreads - 1) sh.pss[kQrMaxGroups] = ld_dev(&part[kPartAlpha]);
    __syncthreads();
    if (tid == 0) {
        double sig = 0.0;
        for (int q = 0; q < P; ++q) sig = sig + sh.pss[q];
        const double alpha = sh.pss[kQrMaxGroups];
        double tau = 0.0, scal = 1.0, beta = alpha;
        if (sig != 0.0) {
            const double nrm = sqrt(alpha * alpha + sig);
            beta = alpha >= 0.0 ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        sh.sc[0] = tau; sh.sc[1] = scal; sh.sc[2] = beta;
    }
    __syncthreads();
    const double tau = sh.sc[0], scal = sh.sc[1];
    double v[kQrRows];
#pragma unroll
    for (int s = 0; s < kQrRows; ++s) {
        const int i = row0 + s * kQrThreads;
        v[s] = 0.0;
        if (i == J) {
            v[s] = 1.0;
            X[s][0] = sh.sc[2];
        } else if (i > J && i < m) {
            double x = X[s][0];
            if (tau != 0.0) {
                x = x * scal;
                X[s][0] = x;
            }
            v[s] = x;
        }
    }
    // 3. partial dot products of v with the other slots (the columns right of J
    //    for the update, the finished ones for T_b), rows >= J
    if (tau != 0.0) {
        double d[kQrNB];
        d[0] = 0.0;
#pragma unroll
        for (int c = 1; c < kQrNB; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int s = 0; s < kQrRows; ++s) {
                const int i = row0 + s * kQrThreads;
                if (i >= J && i < m) acc = acc + v[s] * X[s][c];
            }
            d[c] = acc;
        }
        const double dl = wave_reduce_scatter<kQrNB>(d, lane);
        if ((lane & (kWave / kQrNB - 1)) == 0) sh.rw[wave][lane / (kWave / kQrNB)] = dl;
    }
    __syncthreads();
    if (tau != 0.0 && tid >= 1 && tid < kQrNB)
        st_dev(&part[kPartDot + g * kQrNB + tid], (sh.rw[0][tid] + sh.rw[1][tid]) + (sh.rw[2][tid] + sh.rw[3][tid]));
    if (grid_barrier(a.sync, a.sync + 1, ++epoch, a.spin_limit, false)) return false;
    // 4. sums in group order; the columns right of J; T_b column jj
    if (tau != 0.0)
        for (int e = tid; e < P * kQrNB; e += kQrThreads) sh.pdot[e] = ld_dev(&part[kPartDot + e]);
    __syncthreads();
    if (tid < kQrNB) {
        double sum = 0.0;
        if (tau != 0.0 && tid >= 1)
            for (int q = 0; q < P; ++q) sum = sum + sh.pdot[q * kQrNB + tid];
        sh.dsum[tid] = sum;
    }
    __syncthreads();
    if (tau != 0.0) {
        const int nright = nbw - jj;          // slots 1 .. nright-1 hold the columns right of J
#pragma unroll
        for (int c = 1; c < kQrNB; ++c) {
            if (c < nright) {
                const double t = -tau * sh.dsum[c];
#pragma unroll
                for (int s = 0; s < kQrRows; ++s) {
                    const int i = row0 + s * kQrThreads;
                    if (i >= J && i < m) X[s][c] = X[s][c] + v[s] * t;
                }
            }
        }
    }
    if (tid < jj) {
        double acc = 0.0;
        if (tau != 0.0)
            for (int l = tid; l < jj; ++l) acc = acc + sh.Tb[tid][l] * sh.dsum[kQrNB - jj + l];
        sh.Tb[tid][jj] = -tau * acc;
    }
    if (tid == 0) {
        sh.Tb[jj][jj] = tau;
        if (g == 0) a.tau[J] = tau;
    }
    __syncthreads();             // rw, sc, pss, pdot, dsum and Tb are rewritten by the next column
    qr_rotate(X);
    return true;
}

__global__ __launch_bounds__(kQrThreads) void qr_panel_kernel(QrPanelArgs a) {
    __shared__ QrShared sh;
    auto& red = sh.red;
    auto& Tb = sh.Tb;
    auto& Ys = sh.Ys;
    auto& Us = sh.Us;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int g = blockIdx.x, P = gridDim.x;
    const int m = a.m, w = a.w;
    const long long lda = a.lda;
    double* __restrict__ A = a.A;
    const int row0 = g * kQrGroupRows + tid;
    unsigned epoch = 0;
    if (g == 0 && tid == 0 && a.sync_next) a.sync_next[0] = 0u;
    double* part = a.part;
    const int ww = kQrNB * w;                      // entries of one group's partial W

    for (int cb = 0; cb < w; cb += kQrNB) {
        const int nbw = min(kQrNB, w - cb);
        double X[kQrRows][kQrNB];
#pragma unroll
        for (int s = 0; s < kQrRows; ++s) {
            const long long r = min(row0 + s * kQrThreads, m - 1);
#pragma unroll
            for (int c = 0; c < kQrNB; ++c) X[s][c] = A[r + (long long)min(cb + c, w - 1) * lda];
        }
        Tb[tid / kQrNB][tid % kQrNB] = 0.0;        // 256 threads = 16 x 16 entries

        {
            const QrPos pos{tid, lane, wave, g, P, row0};
#pragma unroll 1
            for (int jj = 0; jj < nbw; ++jj)
                if (!qr_column(X, sh, a, pos, cb, nbw, jj, epoch)) return;
#pragma unroll 1
            for (int jj = nbw; jj < kQrNB; ++jj) qr_rotate(X);   // slot c holds column cb + c again
        }

        // the inner block's R and V back to memory; then X <- V_b (unit lower, 0 outside)
#pragma unroll
        for (int s = 0; s < kQrRows; ++s) {
            const int i = row0 + s * kQrThreads;
#pragma unroll
            for (int c = 0; c < kQrNB; ++c) {
                if (i < m && c < nbw) A[i + (long long)(cb + c) * lda] = X[s][c];
                const int d = cb + c;
                X[s][c] = (c >= nbw || i >= m || i < d) ? 0.0 : (i == d ? 1.0 : X[s][c]);
            }
        }
        if (g == 0) {
            const int r = tid / kQrNB, c = tid % kQrNB;
            if (r <= c && c < nbw) a.T[(cb + r) + (long long)(cb + c) * w] = Tb[r][c];
        }
        if (w == nbw) break;                 // a single inner block: nothing outside it

        // 5. partial W[:, c] = V_b^T A[:, c] over the group's rows, for the panel
        //    columns left (c < cb) and right (c >= cb + 16) of the block, in
        //    chunks of kQrWc columns (value cc * 16 + l of a chunk ends in lanes
        //    (64 / kQrWv) * (cc * 16 + l) after the reduce-scatter)
        double* Wp = part + kPartW + (size_t)g * ww;
        const int nleft = cb / kQrWc, nright = (w - (cb + kQrNB) + kQrWc - 1) / kQrWc;
        const int nch = nleft + (nright > 0 ? nright : 0);
        auto chunk_col = [&](int ch) { return ch < nleft ? kQrWc * ch : cb + kQrNB + kQrWc * (ch - nleft); };
        // the next chunk's loads are in flight while the current one is reduced
        double xn[kQrRows][kQrWc];
        auto load_chunk = [&](int ch) {
            const int c0 = chunk_col(ch);
#pragma unroll
            for (int s = 0; s < kQrRows; ++s) {
                const long long r = min(row0 + s * kQrThreads, m - 1);
#pragma unroll
                for (int cc = 0; cc < kQrWc; ++cc) xn[s][cc] = A[r + (long long)min(c0 + cc, w - 1) * lda];
            }
        };
        if (nch > 0) load_chunk(0);
        for (int r0 = 0; r0 < nch; r0 += kQrRound) {
            const int rn = min(kQrRound, nch - r0);
            for (int k = 0; k < rn; ++k) {
                double x[kQrRows][kQrWc];
#pragma unroll
                for (int s = 0; s < kQrRows; ++s)
#pragma unroll
                    for (int cc = 0; cc < kQrWc; ++cc) x[s][cc] = xn[s][cc];
                if (r0 + k + 1 < nch) load_chunk(r0 + k + 1);
                double acc[kQrWv];
#pragma unroll
                for (int cc = 0; cc < kQrWc; ++cc)
#pragma unroll
                    for (int l = 0; l < kQrNB; ++l) {
                        double t = 0.0;
#pragma unroll
                        for (int s = 0; s < kQrRows; ++s) t = t + X[s][l] * x[s][cc];
                        acc[cc * kQrNB + l] = t;
                    }
                const double tot = wave_reduce_scatter<kQrWv>(acc, lane);
                if ((lane & (kWave / kQrWv - 1)) == 0) red[wave][k][lane / (kWave / kQrWv)] = tot;
            }
            __syncthreads();
            for (int e = tid; e < rn * kQrWv; e += kQrThreads) {
                const int k = e / kQrWv, ev = e % kQrWv;
                const int c = chunk_col(r0 + k) + ev / kQrNB;
                if (c < w)
                    Wp[(ev % kQrNB) + kQrNB * c] = (red[0][k][ev] + red[1][k][ev]) + (red[2][k][ev] + red[3][k][ev]);
            }
            __syncthreads();
        }
        if (grid_barrier(a.sync, a.sync + 1, ++epoch, a.spin_limit)) return;
        // 6. the P partials summed in group order, entries spread over all groups
        for (int e = g * kQrThreads + tid; e < ww; e += kQrThreads * P) {
            const int c = e / kQrNB;
            if (c >= cb && c < cb + kQrNB) continue;
            double sum = 0.0;
#pragma unroll 8
            for (int q = 0; q < P; ++q) sum = sum + part[kPartW + (size_t)q * ww + e];
            part[kPartWs + e] = sum;
        }
        if (grid_barrier(a.sync, a.sync + 1, ++epoch, a.spin_limit)) return;
        // 7. Y = T_b^T W for the columns right of the block (then their
        //    update) and U = (V^T V_b) T_b for the columns left of it; one
        //    column of W per thread
        const double* Ws = part + kPartWs;
        const int c1 = cb + kQrNB;
        for (int c = tid; c < w; c += kQrThreads) {
            if (c >= cb && c < c1) continue;
            double wv[kQrNB];
#pragma unroll
            for (int p = 0; p < kQrNB; ++p) wv[p] = Ws[p + kQrNB * c];
            if (c >= c1) {
#pragma unroll
                for (int l = 0; l < kQrNB; ++l) {
                    double acc = 0.0;
#pragma unroll
                    for (int p = 0; p <= l; ++p) acc = acc + Tb[p][l] * wv[p];
                    Ys[l][c - c1] = acc;
                }
            } else {
#pragma unroll
                for (int q = 0; q < kQrNB; ++q) {
                    double acc = 0.0;
#pragma unroll
                    for (int l = 0; l <= q; ++l) acc = acc + wv[l] * Tb[l][q];
                    Us[c][q] = acc;
                }
            }
        }
        __syncthreads();
        {
            // the update, 4 columns at a time, the next 4 loaded during the current
            double yn[kQrRows][4];
            auto load_cols = [&](int c00) {
#pragma unroll
                for (int s = 0; s < kQrRows; ++s) {
                    const long long r = min(row0 + s * kQrThreads, m - 1);
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) yn[s][cc] = A[r + (long long)min(c00 + cc, w - 1) * lda];
                }
            };
            if (c1 < w) load_cols(c1);
            for (int c00 = c1; c00 < w; c00 += 4) {
                double x[kQrRows][4];
#pragma unroll
                for (int s = 0; s < kQrRows; ++s)
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) x[s][cc] = yn[s][cc];
                if (c00 + 4 < w) load_cols(c00 + 4);
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) {
                    const int c = c00 + cc;
                    if (c < w) {
#pragma unroll
                        for (int s = 0; s < kQrRows; ++s) {
                            const int i = row0 + s * kQrThreads;
                            double t = 0.0;
#pragma unroll
                            for (int l = 0; l < kQrNB; ++l) t = t + X[s][l] * Ys[l][c - c1];
                            if (i >= cb && i < m) A[i + (long long)c * lda] = x[s][cc] - t;
                        }
                    }
                }
            }
        }
        // T[0:cb, block] = -T[0:cb, 0:cb] U: T's rows in runs of 64, one run per
        // wave (lane = row, so each column of T is read coalesced), all 16
        // block columns per lane; the sum over c runs in column order
        for (int run = g * kQrWaves + wave; run * kWave < cb; run += P * kQrWaves) {
            const int r = run * kWave + lane;
            const int rr = min(r, cb - 1);
            double acc[kQrNB];
#pragma unroll
            for (int q = 0; q < kQrNB; ++q) acc[q] = 0.0;
#pragma unroll 16
            for (int c = run * kWave; c < cb; ++c) {
                const double tv = a.T[rr + (long long)c * w];
                const double t = r <= c ? tv : 0.0;          // T is upper triangular
#pragma unroll
                for (int q = 0; q < kQrNB; ++q) acc[q] = acc[q] + t * Us[c][q];
            }
            if (r < cb) {
#pragma unroll
                for (int q = 0; q < kQrNB; ++q)
                    if (q < nbw) a.T[r + (long long)(cb + q) * w] = -acc[q];
            }
        }
        __syncthreads();                     // Tb, Ys and Us are rewritten by the next block
    }
}

// V of the panel as two explicit operands for the trailing update: Vw (m x w,
// column-major, ld m) and its transpose VT (w x m, ld w), unit lower; and
// TT = T^T (w x w, ld w, zero above the diagonal).
__global__ __launch_bounds__(256) void qr_prep_kernel(const double* __restrict__ A, long long lda, int m, int w,
                                                      const double* __restrict__ T, double* __restrict__ Vw,
                                                      double* __restrict__ VT, double* __restrict__ TT) {
    const long long total = (long long)m * w;
    for (long long e = blockIdx.x * 256ll + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
        const int i = (int)(e % m);
        const int c = (int)(e / m);
        const double v = i > c ? A[i + (long long)c * lda] : (i == c ? 1.0 : 0.0);
        Vw[i + (long long)c * m] = v;
        VT[c + (long long)i * w] = v;
        if (i < w) TT[i + (long long)c * w] = i >= c ? T[c + (long long)i * w] : 0.0;
    }
}

// W = sum over s < S of the k-slices Wp[s * count + e], in s order.
__global__ __launch_bounds__(256) void qr_wsum_kernel(const double* __restrict__ Wp, int S, long long count,
                                                      double* __restrict__ W) {
    for (long long e = blockIdx.x * 256ll + threadIdx.x; e < count; e += (long long)gridDim.x * 256) {
        double acc = Wp[e];
        for (int z = 1; z < S; ++z) acc = acc + Wp[(long long)z * count + e];
        W[e] = acc;
    }
}

inline int grid_for(long long work) {
    long long g = (work + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

int launch_qr_panel(const QrPanelArgs& args, int wgs, hipStream_t stream) {
    if (args.w < 1 || args.w > kQrMaxW || args.m < args.w || wgs < 1 || wgs > kQrMaxGroups) return -1;
    if (wgs != (args.m + kQrThreads * kQrRows - 1) / (kQrThreads * kQrRows)) return -1;
    hipLaunchKernelGGL(qr_panel_kernel, dim3(wgs), dim3(kQrThreads), 0, stream, args);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_qr_prep(const double* A, long long lda, int m, int w, const double* T, double* Vw, double* VT,
                   double* TT, hipStream_t stream) {
    if (m <= 0 || w <= 0 || m < w) return 0;
    hipLaunchKernelGGL(qr_prep_kernel, dim3(grid_for((long long)m * w)), dim3(256), 0, stream, A, lda, m, w, T, Vw,
                       VT, TT);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_qr_wsum(const double* Wp, int S, long long count, double* W, hipStream_t stream) {
    if (S <= 0 || count <= 0) return 0;
    hipLaunchKernelGGL(qr_wsum_kernel, dim3(grid_for(count)), dim3(256), 0, stream, Wp, S, count, W);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace lu
