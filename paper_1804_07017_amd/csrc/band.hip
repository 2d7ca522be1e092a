// Transpose of a column-major FP64 block, for the row panel of the two-sided
// band reduction: the panel's w rows are factored as the columns of their
// transpose by the Householder panel kernel and written back.  64 x 64 tiles
// staged through LDS so that both the reads and the writes are coalesced.
#include "common.hpp"
#include "kernels.hpp"

namespace lu {

namespace {

constexpr int kTile = 64;

__global__ __launch_bounds__(256) void transpose_f64_kernel(const double* __restrict__ src, long long lds, int rows,
                                                            int cols, double* __restrict__ dst, long long ldd) {
    __shared__ double tile[kTile][kTile + 1];
    const int r0 = blockIdx.x * kTile, c0 = blockIdx.y * kTile;
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;    // 64 x 4 threads
    for (int j = ty; j < kTile; j += 4) {
        const int r = r0 + tx, c = c0 + j;
        if (r < rows && c < cols) tile[j][tx] = src[r + (long long)c * lds];
    }
    __syncthreads();
    for (int j = ty; j < kTile; j += 4) {
        const int c = c0 + tx, r = r0 + j;          // dst(c, r) = src(r, c)
        if (r < rows && c < cols) dst[c + (long long)r * ldd] = tile[tx][j];
    }
}

}  // namespace

int launch_transpose_f64(const double* src, long long lds, int rows, int cols, double* dst, long long ldd,
                         hipStream_t stream) {
    if (rows <= 0 || cols <= 0) return 0;
    const int gx = (rows + kTile - 1) / kTile, gy = (cols + kTile - 1) / kTile;
    if (gy > 65535) return -1;
    hipLaunchKernelGGL(transpose_f64_kernel, dim3(gx, gy), dim3(256), 0, stream, src, lds, rows, cols, dst, ldd);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace lu
