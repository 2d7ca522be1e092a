// Householder QR with look-ahead: A = Q R, Q = H_0 H_1 ... with
// H_j = I - tau_j v_j v_j^T (LAPACK geqrf storage: R on and above the
// diagonal, v below it with v_j = 1 implicit).  QR fits the blocked skeleton
// of the paper (Sec. 3.1): per iteration the panel is factored with
// Householder reflectors and their block form Q_k = I - V T V^T (T upper
// triangular) is applied to the trailing matrix, C <- Q_k^T C =
// C - V (T^T (V^T C)); the look-ahead of Sec. 4 applies unchanged.
//
// Panel kernel: one persistent launch of P work-groups (256 threads each),
// thread t of group g owning panel rows g*256 + t + s*256*P (s < 4).  Per
// column j, with two device-wide barriers:
//   1. each group's partial sum of squares below the diagonal -> barrier;
//   2. every group forms the same reflector (beta, tau, 1/(alpha - beta)) from
//      the partials summed in group order, scales its rows of v;
//   3. each group's partial dot products v^T A[:, c] for every other panel
//      column c (rows >= j) -> barrier;
//   4. every group sums them in group order, applies the reflector to its rows
//      of the columns right of j; group 0 stores beta, tau_j and column j of T
//      (T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^T v_j), T[j, j] = tau_j).
// Every element sees a fixed operation order whatever P.
#include "common.hpp"
#include "kernels.hpp"

namespace lu {

namespace {

constexpr int kQrThreads = 256;
constexpr int kQrRows = 4;          // panel rows per thread (the launch has >= m / 1024 groups)
constexpr int kQrMaxW = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__global__ __launch_bounds__(kQrThreads) void qr_panel_kernel(QrPanelArgs a) {
    __shared__ double red[kQrThreads / kWave][kQrMaxW];
    __shared__ double wv[kQrMaxW];
    __shared__ double sc[4];                 // tau, scal, beta
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int g = blockIdx.x, P = gridDim.x;
    const int m = a.m, w = a.w;
    const long long lda = a.lda;
    double* __restrict__ A = a.A;
    const int stride = kQrThreads * P;
    const int row0 = g * kQrThreads + tid;
    unsigned epoch = 0;
    if (g == 0 && tid == 0 && a.sync_next) a.sync_next[0] = 0u;
    double* part1 = a.part;                  // [P]
    double* part3 = a.part + 64;             // [P][w]

    for (int j = 0; j < w; ++j) {
        double* colj = A + (long long)j * lda;
        // 1. partial sum of squares of column j below the diagonal
        double ss = 0.0;
#pragma unroll
        for (int s = 0; s < kQrRows; ++s) {
            const int i = row0 + s * stride;
            if (i > j && i < m) {
                const double x = colj[i];
                ss = ss + x * x;
            }
        }
        ss = wave_sum(ss);
        if (lane == 0) red[wave][0] = ss;
        __syncthreads();
        if (tid == 0) part1[g] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
        if (grid_barrier(a.sync, a.sync + 1, ++epoch, a.spin_limit)) return;
        // 2. the reflector, identical in every group
        if (tid == 0) {
            double sig = 0.0;
            for (int q = 0; q < P; ++q) sig = sig + part1[q];
            const double alpha = colj[j];
            double tau = 0.0, scal = 1.0, beta = alpha;
            if (sig != 0.0) {
                const double nrm = sqrt(alpha * alpha + sig);
                beta = alpha >= 0.0 ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            sc[0] = tau; sc[1] = scal; sc[2] = beta;
        }
        __syncthreads();
        const double tau = sc[0], scal = sc[1];
        double v[kQrRows];
#pragma unroll
        for (int s = 0; s < kQrRows; ++s) {
            const int i = row0 + s * stride;
            v[s] = 0.0;
            if (i == j) v[s] = 1.0;
            else if (i > j && i < m) {
                double x = colj[i];
                if (tau != 0.0) {
                    x = x * scal;
                    colj[i] = x;
                }
                v[s] = x;
            }
        }
        // 3. partial dot products v^T A[:, c] (rows >= j) for every panel column c != j
        if (tau != 0.0) {
            for (int c = 0; c < w; ++c) {
                if (c == j) continue;
                const double* colc = A + (long long)c * lda;
                double acc = 0.0;
#pragma unroll
                for (int s = 0; s < kQrRows; ++s) {
                    const int i = row0 + s * stride;
                    if (i >= j && i < m) acc = acc + v[s] * colc[i];
                }
                acc = wave_sum(acc);
                if (lane == 0) red[wave][c] = acc;
            }
        }
        __syncthreads();
        if (tau != 0.0) {
            for (int c = tid; c < w; c += kQrThreads)
                if (c != j) part3[(size_t)g * kQrMaxW + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
        }
        if (grid_barrier(a.sync, a.sync + 1, ++epoch, a.spin_limit)) return;
        // 4. sums in group order; the reflector applied to the columns right of j
        if (tau != 0.0) {
            for (int c = tid; c < w; c += kQrThreads) {
                double sum = 0.0;
                if (c != j)
                    for (int q = 0; q < P; ++q) sum = sum + part3[(size_t)q * kQrMaxW + c];
                wv[c] = sum;
            }
        }
        __syncthreads();
        if (tau != 0.0) {
            for (int c = j + 1; c < w; ++c) {
                double* colc = A + (long long)c * lda;
                const double t = -tau * wv[c];
#pragma unroll
                for (int s = 0; s < kQrRows; ++s) {
                    const int i = row0 + s * stride;
                    if (i >= j && i < m) colc[i] = colc[i] + v[s] * t;
                }
            }
        }
        if (g == 0) {
            // T[0:j, j] = -tau T[0:j, 0:j] s(0:j), s(l) = V[:, l]^T v_j
            double* T = a.T;
            for (int r = tid; r < j; r += kQrThreads) {
                double acc = 0.0;
                if (tau != 0.0)
                    for (int l = r; l < j; ++l) acc = acc + T[r + (long long)l * w] * wv[l];
                T[r + (long long)j * w] = -tau * acc;
            }
            if (tid == 0) {
                T[j + (long long)j * w] = tau;
                a.tau[j] = tau;
                colj[j] = sc[2];
            }
            __threadfence_block();
        }
        __syncthreads();     // wv, sc and red are rewritten by the next column
    }
}

// V of the panel as two explicit operands for the trailing update: Vw (m x w,
// column-major, ld m) and its transpose VT (w x m, ld w), unit lower.
__global__ __launch_bounds__(256) void qr_prep_kernel(const double* __restrict__ A, long long lda, int m, int w,
                                                      double* __restrict__ Vw, double* __restrict__ VT) {
    const long long total = (long long)m * w;
    for (long long e = blockIdx.x * 256ll + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
        const int i = (int)(e % m);
        const int c = (int)(e / m);
        const double v = i > c ? A[i + (long long)c * lda] : (i == c ? 1.0 : 0.0);
        Vw[i + (long long)c * m] = v;
        VT[c + (long long)i * w] = v;
    }
}

// Ym = -T^T W (w x nc, both column-major with ld w); T upper triangular.
__global__ __launch_bounds__(256) void qr_tmul_kernel(const double* __restrict__ T, int w, const double* __restrict__ W,
                                                      int nc, double* __restrict__ Ym) {
    const long long total = (long long)w * nc;
    for (long long e = blockIdx.x * 256ll + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
        const int r = (int)(e % w);
        const long long col = e / w;
        double acc = 0.0;
        for (int l = 0; l <= r; ++l) acc = acc + T[l + (long long)r * w] * W[l + col * w];
        Ym[r + col * w] = -acc;
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
    if (args.w < 1 || args.w > kQrMaxW || args.m < args.w || wgs < 1 || wgs > 64) return -1;
    if ((long long)wgs * kQrThreads * kQrRows < args.m) return -1;
    hipLaunchKernelGGL(qr_panel_kernel, dim3(wgs), dim3(kQrThreads), 0, stream, args);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_qr_prep(const double* A, long long lda, int m, int w, double* Vw, double* VT, hipStream_t stream) {
    if (m <= 0 || w <= 0) return 0;
    hipLaunchKernelGGL(qr_prep_kernel, dim3(grid_for((long long)m * w)), dim3(256), 0, stream, A, lda, m, w, Vw, VT);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_qr_tmul(const double* T, int w, const double* W, int nc, double* Ym, hipStream_t stream) {
    if (w <= 0 || nc <= 0) return 0;
    hipLaunchKernelGGL(qr_tmul_kernel, dim3(grid_for((long long)w * nc)), dim3(256), 0, stream, T, w, W, nc, Ym);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace lu
