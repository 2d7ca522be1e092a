// The schedule selector's network on the GPU: forward, backward and Adam.
//
// 4 inputs -> 32 ReLU hidden units -> 10 logits in three softmax heads
// (block size: 4 classes, look-ahead depth: 3, panel CU share: 3).  Loss: the
// batch mean of the summed per-head cross-entropies.  Parameters in one flat
// FP32 vector: W1 (32x4 row-major), b1[32], W2 (10x32 row-major), b2[10].
// One work-group runs a whole training job: each thread owns one training row
// for the forward/backward pass; gradients are reduced over rows in a fixed
// order, so a run is deterministic.
#include "common.hpp"
#include "kernels.hpp"

namespace lu {

namespace {

constexpr int kIn = 4, kHid = 32, kOut = 10, kMaxBatch = 256;
constexpr int kParams = kHid * kIn + kHid + kOut * kHid + kOut;   // 490
constexpr int oW1 = 0, ob1 = kHid * kIn, oW2 = ob1 + kHid, ob2 = oW2 + kOut * kHid;
__constant__ int kHeadLo[3] = {0, 4, 7};
__constant__ int kHeadHi[3] = {4, 7, 10};

__device__ void forward_row(const float* th, const float* x, float* a, float* h, float* z) {
    for (int u = 0; u < kHid; ++u) {
        float s = th[ob1 + u];
        for (int i = 0; i < kIn; ++i) s += th[oW1 + u * kIn + i] * x[i];
        a[u] = s;
        h[u] = s > 0.f ? s : 0.f;
    }
    for (int o = 0; o < kOut; ++o) {
        float s = th[ob2 + o];
        for (int u = 0; u < kHid; ++u) s += th[oW2 + o * kHid + u] * h[u];
        z[o] = s;
    }
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* theta, const float* X, int batch,
                                                          float* logits) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= batch) return;
    float a[kHid], h[kHid], z[kOut];
    forward_row(theta, X + r * kIn, a, h, z);
    for (int o = 0; o < kOut; ++o) logits[r * kOut + o] = z[o];
}

__global__ __launch_bounds__(256) void mlp_train_kernel(float* theta, float* mom, float* vel, const float* X,
                                                        const int* Y, int batch, int epochs, float lr, int t0,
                                                        float* loss_out, float* grad_out, int update) {
    __shared__ float s_th[kParams];
    __shared__ float s_x[kMaxBatch][kIn];
    __shared__ float s_h[kMaxBatch][kHid + 1];
    __shared__ float s_da[kMaxBatch][kHid + 1];
    __shared__ float s_dz[kMaxBatch][kOut];
    __shared__ float s_loss[kMaxBatch];
    const int tid = threadIdx.x;
    for (int p = tid; p < kParams; p += 256) s_th[p] = theta[p];
    for (int e = tid; e < batch * kIn; e += 256) s_x[e / kIn][e % kIn] = X[e];
    __syncthreads();
    const float inv_b = 1.f / (float)batch;
    for (int ep = 0; ep < epochs; ++ep) {
        if (tid < batch) {
            float a[kHid], h[kHid], z[kOut];
            forward_row(s_th, s_x[tid], a, h, z);
            float dz[kOut];
            float l = 0.f;
            for (int hd = 0; hd < 3; ++hd) {
                const int lo = kHeadLo[hd], hi = kHeadHi[hd];
                float mx = z[lo];
                for (int o = lo + 1; o < hi; ++o) mx = fmaxf(mx, z[o]);
                float se = 0.f;
                for (int o = lo; o < hi; ++o) se += expf(z[o] - mx);
                const float lse = mx + logf(se);
                const int y = lo + Y[tid * 3 + hd];
                l += lse - z[y];
                for (int o = lo; o < hi; ++o) dz[o] = (expf(z[o] - lse) - (o == y ? 1.f : 0.f)) * inv_b;
            }
            s_loss[tid] = l;
            for (int o = 0; o < kOut; ++o) s_dz[tid][o] = dz[o];
            for (int u = 0; u < kHid; ++u) {
                float dh = 0.f;
                for (int o = 0; o < kOut; ++o) dh += dz[o] * s_th[oW2 + o * kHid + u];
                s_da[tid][u] = a[u] > 0.f ? dh : 0.f;
                s_h[tid][u] = h[u];
            }
        }
        __syncthreads();
        if (tid == 0 && loss_out) {
            float L = 0.f;
            for (int r = 0; r < batch; ++r) L += s_loss[r];
            loss_out[ep] = L * inv_b;
        }
        // gradient of parameter p (fixed reduction order over rows) and the Adam step
        for (int p = tid; p < kParams; p += 256) {
            float g = 0.f;
            if (p < ob1) {
                const int u = p / kIn, i = p % kIn;
                for (int r = 0; r < batch; ++r) g += s_da[r][u] * s_x[r][i];
            } else if (p < oW2) {
                const int u = p - ob1;
                for (int r = 0; r < batch; ++r) g += s_da[r][u];
            } else if (p < ob2) {
                const int o = (p - oW2) / kHid, u = (p - oW2) % kHid;
                for (int r = 0; r < batch; ++r) g += s_dz[r][o] * s_h[r][u];
            } else {
                const int o = p - ob2;
                for (int r = 0; r < batch; ++r) g += s_dz[r][o];
            }
            if (grad_out) grad_out[p] = g;
            if (update) {
                const int t = t0 + ep + 1;
                const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
                const float m = b1 * mom[p] + (1.f - b1) * g;
                const float v = b2 * vel[p] + (1.f - b2) * g * g;
                mom[p] = m;
                vel[p] = v;
                const float mh = m / (1.f - powf(b1, (float)t));
                const float vh = v / (1.f - powf(b2, (float)t));
                s_th[p] = s_th[p] - lr * mh / (sqrtf(vh) + eps);
            }
        }
        __syncthreads();
    }
    for (int p = tid; p < kParams; p += 256) theta[p] = s_th[p];
}

}  // namespace

int launch_mlp_forward(const float* theta, const float* X, int batch, float* logits, hipStream_t stream) {
    if (batch <= 0) return 0;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((batch + 255) / 256), dim3(256), 0, stream, theta, X, batch, logits);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mlp_train(float* theta, float* m, float* v, const float* X, const int* Y, int batch, int epochs, float lr,
                     int t0, float* loss_out, float* grad_out, int update, hipStream_t stream) {
    if (batch <= 0 || batch > kMaxBatch) return -1;
    hipLaunchKernelGGL(mlp_train_kernel, dim3(1), dim3(256), 0, stream, theta, m, v, X, Y, batch, epochs, lr, t0,
                       loss_out, grad_out, update);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace lu
