// gfx950 matrix-core helpers shared by the GEMM and TRSM kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace lu {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// 16x16 MFMA with 4-deep k (FP64 / FP32): D = A B + C, where lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Accumulator type and output lane
// layout: lane l, register r holds D[row(l / 16, r)][l % 16] with
//   v_mfma_f64_16x16x4f64:   row = l/16 + 4r   (measured on gfx950)
//   v_mfma_f32_16x16x4f32:   row = 4(l/16) + r
// The kernels feed the transposed problem (first operand = the right factor
// transposed), so D's rows run along the result's columns and a lane holds 16
// consecutive ROWS of one column: coalesced for column-major storage.
template <typename T> struct Acc;
template <> struct Acc<double> {
    typedef v4d type;
    static __device__ __forceinline__ int col(int lg, int r) { return lg + 4 * r; }
};
template <> struct Acc<float> {
    typedef v4f type;
    static __device__ __forceinline__ int col(int lg, int r) { return 4 * lg + r; }
};

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

}  // namespace lu
