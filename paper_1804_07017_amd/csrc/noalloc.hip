// lu_solve_noalloc: lu_solve_ex with its scratch memory (the per-chunk
// interchange lists, the triangular solves' ready flags and their error word)
// in one file-scope device array instead of library-allocated buffers, for
// callers that cannot allocate (graph capture, tight serving loops).  The
// kernels are the ones lu_solve_ex launches.
//
// Host code never passes `scratch` itself to a kernel: in host code the name
// is a stand-in, not a device address.  The device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/lu.h"
#include "../../include/lu_kernels.h"
#include "kernels.hpp"

namespace lu {

namespace {

constexpr int kChunkW = 512;                      // rows per interchange chunk, as lu_solve_ex
constexpr int kMaxDevices = 64;

// layout: [0, 256) error word; then the ready flags; then the interchange lists
constexpr size_t kErrBytes = 256;
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t flag_bytes(int n) { return align256((size_t)((n + kTrsvRows - 1) / kTrsvRows) * sizeof(int)); }
constexpr size_t moves_bytes(int n) { return (size_t)((n + kChunkW - 1) / kChunkW) * kMovesLen * sizeof(int); }
constexpr size_t kScratchBytes = kErrBytes + flag_bytes(LU_NOALLOC_MAX_N) + moves_bytes(LU_NOALLOC_MAX_N);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

unsigned char* g_scratch[kMaxDevices];            // device address of `scratch`, per device
long long g_spin[kMaxDevices];                    // wait bound of the triangular solves, per device

// Device address of this device's copy of `scratch` and the solves' wait
// bound (about 2 s of the device wall clock), taken on the first call on the
// device.  No allocation.
int setup(int dev) {
    if (g_scratch[dev]) return 0;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LU_ERR_HIP;
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate_khz <= 0)
        rate_khz = 100000;
    g_spin[dev] = (long long)rate_khz * 1000ll * 2;
    g_scratch[dev] = static_cast<unsigned char*>(p);
    return 0;
}

}  // namespace

}  // namespace lu

extern "C" {

int lu_solve_noalloc(int n, int nrhs, const double* LU, int lda, const int* ipiv, double* B, int ldb,
                     hipStream_t stream) {
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (!LU && n > 0) return -3;
    if (lda < std::max(1, n)) return -4;
    if (!ipiv && n > 0) return -5;
    if (!B && n > 0 && nrhs > 0) return -6;
    if (ldb < std::max(1, n)) return -7;
    if (n > LU_NOALLOC_MAX_N) return LU_ERR_UNSUPPORTED;
    if (n == 0 || nrhs == 0) return 0;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= lu::kMaxDevices) return LU_ERR_HIP;
    if (int rc = lu::setup(dev)) return rc;
    unsigned char* base = lu::g_scratch[dev];
    unsigned* err = reinterpret_cast<unsigned*>(base);
    int* flags = reinterpret_cast<int*>(base + lu::kErrBytes);
    int* mv = reinterpret_cast<int*>(base + lu::kErrBytes + lu::flag_bytes(n));
    const long long spin = lu::g_spin[dev];
    // the array keeps the previous call's contents: the error word and the
    // flags start at zero (fill kernels, not memset nodes), the lists are
    // written whole by launch_chunk_moves
    if (lu::launch_fill_zero(base, lu::kErrBytes + lu::flag_bytes(n), stream)) return LU_ERR_HIP;
    if (lu::launch_chunk_moves(ipiv, n, lu::kChunkW, mv, stream)) return LU_ERR_HIP;
    if (lu::launch_apply_chunk_moves<double>(B, ldb, n, nrhs, lu::kChunkW, mv, stream)) return LU_ERR_HIP;
    int epoch = 0;
    for (int c = 0; c < nrhs; ++c) {
        double* x = B + (long long)c * ldb;
        if (epoch > 0x3ffffff0) {                  // flags back to zero before the epoch wraps
            if (lu::launch_fill_zero(flags, lu::flag_bytes(n), stream)) return LU_ERR_HIP;
            epoch = 0;
        }
        if (lu::launch_trsv_lower_unit<double>(LU, lda, n, x, flags, ++epoch, err, spin, stream)) return LU_ERR_HIP;
        if (lu::launch_trsv_upper<double>(LU, lda, n, x, flags, ++epoch, err, spin, stream)) return LU_ERR_HIP;
    }
    return 0;
}

}  // extern "C"
