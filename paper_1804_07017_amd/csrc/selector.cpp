// Learned schedule selector: weights, features, inference and training entry
// points.  The network itself runs in mlp.hip.
//
// Features of (n, precision): (log2 n - 14) / 3 and a one-hot of
// {FP64, FP32, mixed (FP16 or BF16)}.  Heads: b in {64,128,256,512},
// look-ahead depth in {0,1,2}, panel CU share in {8,16,32}.  The prediction
// is used only for n within [n_min/2, 2 n_max] of the training sizes; outside
// that range, or without weights, the fixed default applies.
#include "selector.hpp"

#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>

#include "../../include/lu.h"
#include "kernels.hpp"

namespace lu {

namespace {
constexpr int kParams = 490;
constexpr char kMagic[8] = {'L', 'U', 'S', 'E', 'L', '0', '0', '1'};
const int kB[4] = {64, 128, 256, 512};
const int kP[3] = {8, 16, 32};

struct Sel {
    bool loaded = false;
    bool tried_default = false;
    float theta[kParams];
    int n_min = 0, n_max = 0;
    std::map<long long, lu_schedule_t> cache;
    // device copies
    float* d_theta = nullptr;
    float* d_m = nullptr;
    float* d_v = nullptr;
    int adam_t = 0;
} g;

void features(int n, int prec, float* x) {
    x[0] = (std::log2((float)n) - 14.f) / 3.f;
    x[1] = prec == LU_FP64 ? 1.f : 0.f;
    x[2] = prec == LU_FP32 ? 1.f : 0.f;
    x[3] = (prec == LU_MIXED_FP16 || prec == LU_MIXED_BF16) ? 1.f : 0.f;
}

int ensure_dev() {
    if (!g.d_theta) {
        if (hipMalloc(&g.d_theta, kParams * sizeof(float)) != hipSuccess) return LU_ERR_NOMEM;
        if (hipMalloc(&g.d_m, kParams * sizeof(float)) != hipSuccess) return LU_ERR_NOMEM;
        if (hipMalloc(&g.d_v, kParams * sizeof(float)) != hipSuccess) return LU_ERR_NOMEM;
        if (hipMemset(g.d_m, 0, kParams * sizeof(float)) != hipSuccess) return LU_ERR_HIP;
        if (hipMemset(g.d_v, 0, kParams * sizeof(float)) != hipSuccess) return LU_ERR_HIP;
    }
    return 0;
}

int load_file(const char* path) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return -1;
    char magic[8];
    int hdr[3];
    float th[kParams];
    int ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
             std::fread(hdr, sizeof(int), 3, f) == 3 && hdr[2] == kParams &&
             std::fread(th, sizeof(float), kParams, f) == (size_t)kParams;
    std::fclose(f);
    if (!ok) return -2;
    if (hdr[0] <= 0 || hdr[1] < hdr[0]) return -2;
    for (int i = 0; i < kParams; ++i)
        if (!std::isfinite(th[i])) return -2;
    std::memcpy(g.theta, th, sizeof th);
    g.n_min = hdr[0];
    g.n_max = hdr[1];
    g.loaded = true;
    g.cache.clear();
    g.adam_t = 0;
    return 0;
}

std::string default_path() {
    Dl_info info;
    if (dladdr((void*)&default_path, &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        size_t s = p.rfind('/');
        if (s != std::string::npos) return p.substr(0, s + 1) + "selector_weights.bin";
    }
    return "selector_weights.bin";
}

void try_default() {
    if (g.tried_default) return;
    g.tried_default = true;
    if (const char* e = std::getenv("LU_SELECTOR_WEIGHTS")) {
        load_file(e);
        return;
    }
    load_file(default_path().c_str());
}

lu_schedule_t fixed_default() { return lu_schedule_t{256, 1, 16, 0}; }

}  // namespace

bool selector_enabled() {
    const char* e = std::getenv("LU_SELECTOR");
    if (e && (std::strcmp(e, "off") == 0 || std::strcmp(e, "0") == 0)) return false;
    try_default();
    return g.loaded;
}

int selector_predict(int n, int prec, lu_schedule_t* out) {
    *out = fixed_default();
    if (!g.loaded) return 1;
    if (n < g.n_min / 2 || (long long)n > 2ll * g.n_max) return 1;
    const int pc = (prec == LU_MIXED_BF16) ? LU_MIXED_FP16 : prec;
    const long long key = ((long long)n << 3) | pc;
    auto it = g.cache.find(key);
    if (it != g.cache.end()) { *out = it->second; return 0; }
    if (ensure_dev()) return 1;
    float x[4];
    features(n, pc, x);
    float* d_x = nullptr;
    float* d_z = nullptr;
    float z[10];
    if (hipMalloc(&d_x, 16 * sizeof(float)) != hipSuccess) return 1;
    d_z = d_x + 4;
    int rc = 1;
    if (hipMemcpy(g.d_theta, g.theta, kParams * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
        hipMemcpy(d_x, x, 4 * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
        launch_mlp_forward(g.d_theta, d_x, 1, d_z, nullptr) == 0 &&
        hipMemcpy(z, d_z, 10 * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess) {
        int ib = 0, id = 4, ip = 7;
        for (int o = 1; o < 4; ++o) if (z[o] > z[ib]) ib = o;
        for (int o = 5; o < 7; ++o) if (z[o] > z[id]) id = o;
        for (int o = 8; o < 10; ++o) if (z[o] > z[ip]) ip = o;
        out->b = kB[ib];
        out->depth = id - 4;
        out->panel_cus = kP[ip - 7];
        g.cache[key] = *out;
        rc = 0;
    }
    hipFree(d_x);
    if (rc) *out = fixed_default();
    return rc;
}

}  // namespace lu

using lu::g;

extern "C" {

int lu_selector_load(const char* path) {
    g.tried_default = true;
    if (!path) {
        g.loaded = false;
        g.cache.clear();
        g.adam_t = 0;
        return 0;
    }
    return lu::load_file(path);
}

int lu_selector_predict(int n, lu_precision_t prec, lu_schedule_t* out) {
    if (n < 1) return -1;
    if (prec < LU_FP64 || prec > LU_MIXED_BF16) return -2;
    if (!out) return -3;
    lu::try_default();
    return lu::selector_predict(n, (int)prec, out);
}

int lu_selector_save(const char* path) {
    if (!path) return -1;
    if (!g.loaded) return -2;
    FILE* f = std::fopen(path, "wb");
    if (!f) return -3;
    int hdr[3] = {g.n_min, g.n_max, lu::kParams};
    bool ok = std::fwrite(lu::kMagic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int), 3, f) == 3 &&
              std::fwrite(g.theta, sizeof(float), lu::kParams, f) == (size_t)lu::kParams;
    std::fclose(f);
    return ok ? 0 : -4;
}

int lu_selector_get_params(float* theta_out, int n_theta) {
    if (!theta_out) return -1;
    if (n_theta < lu::kParams) return -2;
    if (!g.loaded) return 1;
    std::memcpy(theta_out, g.theta, sizeof g.theta);
    return 0;
}

int lu_selector_set_params(const float* theta, int n_theta, int n_min, int n_max) {
    if (!theta) return -1;
    if (n_theta != lu::kParams) return -2;
    if (n_min < 1) return -3;
    if (n_max < n_min) return -4;
    std::memcpy(g.theta, theta, sizeof g.theta);
    g.n_min = n_min;
    g.n_max = n_max;
    g.loaded = true;
    g.tried_default = true;
    g.cache.clear();
    g.adam_t = 0;
    if (lu::ensure_dev()) return LU_ERR_NOMEM;
    if (hipMemset(g.d_m, 0, lu::kParams * sizeof(float)) != hipSuccess) return LU_ERR_HIP;
    if (hipMemset(g.d_v, 0, lu::kParams * sizeof(float)) != hipSuccess) return LU_ERR_HIP;
    return 0;
}

static int run_train(const float* X, const int* Y, int batch, int epochs, float lr, float* loss_out, float* grad_out,
                     int update) {
    // labels index the heads' classes: reject anything outside {0..3} x {0..2} x {0..2}
    static const int kClasses[3] = {4, 3, 3};
    for (int r = 0; r < batch; ++r)
        for (int h = 0; h < 3; ++h)
            if (Y[3 * r + h] < 0 || Y[3 * r + h] >= kClasses[h]) return -2;
    for (int e = 0; e < 4 * batch; ++e)
        if (!std::isfinite(X[e])) return -1;
    if (lu::ensure_dev()) return LU_ERR_NOMEM;
    float* d_x = nullptr;
    int* d_y = nullptr;
    float* d_loss = nullptr;
    float* d_grad = nullptr;
    int rc = 0;
    const int ep_alloc = epochs > 0 ? epochs : 1;
    if (hipMalloc(&d_x, (size_t)batch * 4 * sizeof(float)) != hipSuccess ||
        hipMalloc(&d_y, (size_t)batch * 3 * sizeof(int)) != hipSuccess ||
        hipMalloc(&d_loss, (size_t)ep_alloc * sizeof(float)) != hipSuccess ||
        hipMalloc(&d_grad, lu::kParams * sizeof(float)) != hipSuccess) {
        rc = LU_ERR_NOMEM;
    }
    if (!rc && (hipMemcpy(d_x, X, (size_t)batch * 4 * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(d_y, Y, (size_t)batch * 3 * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(g.d_theta, g.theta, sizeof g.theta, hipMemcpyHostToDevice) != hipSuccess))
        rc = LU_ERR_HIP;
    if (!rc && lu::launch_mlp_train(g.d_theta, g.d_m, g.d_v, d_x, d_y, batch, epochs, lr, g.adam_t, d_loss,
                                    grad_out ? d_grad : nullptr, update, nullptr))
        rc = LU_ERR_HIP;
    if (!rc && hipDeviceSynchronize() != hipSuccess) rc = LU_ERR_HIP;
    if (!rc && update) {
        if (hipMemcpy(g.theta, g.d_theta, sizeof g.theta, hipMemcpyDeviceToHost) != hipSuccess) rc = LU_ERR_HIP;
        g.adam_t += epochs;
        g.cache.clear();
    }
    if (!rc && loss_out &&
        hipMemcpy(loss_out, d_loss, (size_t)ep_alloc * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        rc = LU_ERR_HIP;
    if (!rc && grad_out && hipMemcpy(grad_out, d_grad, lu::kParams * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        rc = LU_ERR_HIP;
    hipFree(d_x);
    hipFree(d_y);
    hipFree(d_loss);
    hipFree(d_grad);
    return rc;
}

int lu_selector_train(const float* X, const int* Y, int batch, int epochs, float lr, int seed, float* loss_out) {
    if (!X) return -1;
    if (!Y) return -2;
    if (batch < 1 || batch > 256) return -3;
    if (epochs < 1) return -4;
    if (!(lr > 0.f)) return -5;
    if (!g.loaded) {
        if (seed < 0) return -6;
        // seeded initialisation: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a 64-bit LCG
        unsigned long long st = 0x9E3779B97F4A7C15ull ^ (unsigned long long)seed;
        auto uni = [&]() {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            return (float)((st >> 11) * (1.0 / 9007199254740992.0));
        };
        for (int p = 0; p < lu::kParams; ++p) {
            const float fan = p < 160 ? 4.f : 32.f;
            g.theta[p] = (2.f * uni() - 1.f) / std::sqrt(fan);
        }
        // training range from the batch's first feature
        float lo = 1e30f, hi = -1e30f;
        for (int r = 0; r < batch; ++r) { lo = std::fmin(lo, X[4 * r]); hi = std::fmax(hi, X[4 * r]); }
        g.n_min = (int)std::lround(std::exp2(3.f * lo + 14.f));
        g.n_max = (int)std::lround(std::exp2(3.f * hi + 14.f));
        g.loaded = true;
        g.adam_t = 0;
        if (lu::ensure_dev()) return LU_ERR_NOMEM;
        hipMemset(g.d_m, 0, lu::kParams * sizeof(float));
        hipMemset(g.d_v, 0, lu::kParams * sizeof(float));
    }
    return run_train(X, Y, batch, epochs, lr, loss_out, nullptr, 1);
}

int lu_selector_grad(const float* X, const int* Y, int batch, float* loss_out, float* grad_out) {
    if (!X) return -1;
    if (!Y) return -2;
    if (batch < 1 || batch > 256) return -3;
    if (!loss_out) return -4;
    if (!grad_out) return -5;
    if (!g.loaded) return 1;
    return run_train(X, Y, batch, 1, 1.f, loss_out, grad_out, 0);
}

}  // extern "C"
