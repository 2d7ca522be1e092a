// Solve entry points: lu_solve / lu_solve_ex (LAPACK getrs semantics with
// the packed factor of lu_factor) and lu_solve_ir (low-precision LU with FP64
// iterative refinement; not part of the paper, the precision axis of this
// library).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/lu.h"
#include "../../include/lu_kernels.h"
#include "kernels.hpp"
#include "state.hpp"

namespace lu {

int factor_impl(int n, void* A, int lda, lu_precision_t prec, int* ipiv, const lu_schedule_t* sched, int* d_info,
                hipStream_t stream);
// dst = (float)A (n x n, leading dimensions lda, ldd) and *out_max = ||A||_inf
// as double bits (atomic max; clear it first), in one pass over A; partial
// holds splits x n doubles.  Defined with the other solve kernels.
int launch_convert_row_abs_sums(const double* A, long long lda, int n, float* dst, long long ldd, double* partial,
                                int splits, double* out_max, hipStream_t stream);

namespace {

constexpr int kChunkW = 512;
constexpr int kSplits = 16;
constexpr double kEps = 1.1102230246251565e-16;   // 2^-53

unsigned* trsv_err(DeviceState* s) { return s->sync + 4; }

// P x then L^-1 then U^-1 on each of nrhs columns, with the factor in type T.
template <typename T>
int solve_with_factor(DeviceState* s, int n, int nrhs, const T* LU, long long lda, const int* ipiv, T* X,
                      long long ldx, hipStream_t stream, bool moves_ready) {
    int rc;
    const int nchunks = (n + kChunkW - 1) / kChunkW;
    if ((rc = ensure(s->solve_moves, (size_t)nchunks * kMovesLen * sizeof(int)))) return rc;
    const int nblk = (n + trsv_block_rows() - 1) / trsv_block_rows();
    if (s->flags.bytes < (size_t)nblk * sizeof(int)) {
        if ((rc = ensure(s->flags, (size_t)nblk * sizeof(int)))) return rc;
        LU_HIP(hipMemset(s->flags.ptr, 0, s->flags.bytes));
        s->trsv_epoch = 0;
    }
    int* mv = reinterpret_cast<int*>(s->solve_moves.ptr);
    if (!moves_ready && launch_chunk_moves(ipiv, n, kChunkW, mv, stream)) return LU_ERR_HIP;
    if (launch_apply_chunk_moves<T>(X, ldx, n, nrhs, kChunkW, mv, stream)) return LU_ERR_HIP;
    int* flags = reinterpret_cast<int*>(s->flags.ptr);
    for (int c = 0; c < nrhs; ++c) {
        T* x = X + (long long)c * ldx;
        if (s->trsv_epoch > 0x3ffffff0) {
            if (launch_fill_zero(s->flags.ptr, s->flags.bytes, stream)) return LU_ERR_HIP;
            s->trsv_epoch = 0;
        }
        if (launch_trsv_lower_unit<T>(LU, lda, n, x, flags, ++s->trsv_epoch, trsv_err(s), s->spin_limit, stream))
            return LU_ERR_HIP;
        if (launch_trsv_upper<T>(LU, lda, n, x, flags, ++s->trsv_epoch, trsv_err(s), s->spin_limit, stream))
            return LU_ERR_HIP;
    }
    return 0;
}

int read_err(DeviceState* s, hipStream_t stream) {
    unsigned e = 0;
    LU_HIP(hipMemcpyAsync(&e, trsv_err(s), sizeof(unsigned), hipMemcpyDeviceToHost, stream));
    LU_HIP(hipStreamSynchronize(stream));
    if (e) {
        LU_HIP(hipMemset(trsv_err(s), 0, sizeof(unsigned)));
        return LU_ERR_BARRIER;
    }
    return 0;
}

double bits_to_double(unsigned long long b) {
    double d;
    std::memcpy(&d, &b, sizeof d);
    return d;
}

// ||v||_inf of a device FP64 vector, read back to the host (synchronises).
int dev_amax(DeviceState* s, const double* v, int n, hipStream_t stream, double* out) {
    unsigned long long* w = reinterpret_cast<unsigned long long*>(s->ir_norms.ptr) + 7;
    if (launch_fill_zero(w, sizeof(*w), stream)) return LU_ERR_HIP;
    if (launch_amax(v, n, w, stream)) return LU_ERR_HIP;
    unsigned long long h = 0;
    LU_HIP(hipMemcpyAsync(&h, w, sizeof h, hipMemcpyDeviceToHost, stream));
    LU_HIP(hipStreamSynchronize(stream));
    *out = bits_to_double(h);
    return 0;
}

// ||u||_inf and ||v||_inf with one read-back (one synchronisation).
int dev_amax2(DeviceState* s, const double* u, const double* v, int n, hipStream_t stream, double* out_u,
              double* out_v) {
    unsigned long long* w = reinterpret_cast<unsigned long long*>(s->ir_norms.ptr) + 8;
    if (launch_fill_zero(w, 2 * sizeof(*w), stream)) return LU_ERR_HIP;
    if (launch_amax(u, n, w, stream)) return LU_ERR_HIP;
    if (launch_amax(v, n, w + 1, stream)) return LU_ERR_HIP;
    unsigned long long h[2] = {0, 0};
    LU_HIP(hipMemcpyAsync(h, w, sizeof h, hipMemcpyDeviceToHost, stream));
    LU_HIP(hipStreamSynchronize(stream));
    *out_u = bits_to_double(h[0]);
    *out_v = bits_to_double(h[1]);
    return 0;
}

// Outcome of a factorization enqueued on `stream` with the library's INFO
// word: waits for it, returns LU_ERR_BARRIER if one of its panel barriers
// timed out (the error words are cleared for the next call), else 0 with
// LAPACK INFO in *info.
int factor_status(DeviceState* s, hipStream_t stream, int* info) {
    int h = 0;
    unsigned e[4] = {0, 0, 0, 0};
    LU_HIP(hipMemcpyAsync(&h, s->info, sizeof(int), hipMemcpyDeviceToHost, stream));
    LU_HIP(hipMemcpyAsync(e, s->sync, 4 * sizeof(unsigned), hipMemcpyDeviceToHost, stream));
    LU_HIP(hipStreamSynchronize(stream));
    *info = h;
    if (e[1] || e[3]) {
        if (launch_fill_zero(s->sync + 1, sizeof(unsigned), stream)) return LU_ERR_HIP;
        if (launch_fill_zero(s->sync + 3, sizeof(unsigned), stream)) return LU_ERR_HIP;
        LU_HIP(hipStreamSynchronize(stream));
        return LU_ERR_BARRIER;
    }
    return 0;
}

// FP64 factor of a copy of A and a plain solve; used for LU_FP64 and as the
// fallback.  A singular FP64 factor (INFO > 0) is reported in *info and
// leaves X unsolved.
int fp64_path(DeviceState* s, int n, int nrhs, const double* A, long long lda, const double* B, long long ldb,
              double* X, long long ldx, hipStream_t stream, int* info) {
    int rc;
    if ((rc = ensure(s->ir_a64, (size_t)n * n * sizeof(double)))) return rc;
    if ((rc = ensure(s->ir_ipiv, (size_t)n * sizeof(int)))) return rc;
    double* A64 = reinterpret_cast<double*>(s->ir_a64.ptr);
    int* ipiv = reinterpret_cast<int*>(s->ir_ipiv.ptr);
    if (launch_copy_f64(A, lda, A64, n, n, n, stream)) return LU_ERR_HIP;
    if ((rc = factor_impl(n, A64, n, LU_FP64, ipiv, nullptr, nullptr, stream))) return rc;
    if ((rc = factor_status(s, stream, info))) return rc;
    if (*info != 0) return 0;
    if (launch_copy_f64(B, ldb, X, ldx, n, nrhs, stream)) return LU_ERR_HIP;
    if ((rc = solve_with_factor<double>(s, n, nrhs, A64, n, ipiv, X, ldx, stream, false))) return rc;
    return read_err(s, stream);
}

// HPL residual of column c: ||A x - b|| / (eps (||A|| ||x|| + ||b||) n), with
// ||b|| given (the caller has it from the input check)
int hpl_resid(DeviceState* s, int n, const double* A, long long lda, const double* b, const double* x, double anorm,
              double bn, hipStream_t stream, double* out) {
    double* r = reinterpret_cast<double*>(s->ir_r.ptr);
    double* part = reinterpret_cast<double*>(s->partial.ptr);
    if (launch_residual(A, lda, n, x, b, r, part, kSplits, stream)) return LU_ERR_HIP;
    double rn, xn;
    int rc;
    if ((rc = dev_amax2(s, r, x, n, stream, &rn, &xn))) return rc;
    const double denom = kEps * (anorm * xn + bn) * (double)n;
    *out = denom > 0 ? rn / denom : (rn == 0 ? 0.0 : INFINITY);
    if (!std::isfinite(rn) || !std::isfinite(xn)) *out = NAN;
    return 0;
}

}  // namespace

int ir_outcome(int fp64_info, int fell_back, double resid) {
    if (fp64_info != 0) return LU_ERR_SINGULAR;
    if (std::isnan(resid)) return LU_ERR_NONFINITE;
    if (!(resid <= 16.0)) return LU_IR_RESID_HIGH;
    return fell_back ? LU_IR_FELL_BACK : LU_IR_OK;
}

int solve_ir_impl(int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X, int ldx,
                  lu_precision_t prec, int max_iter, int* iters_out, double* resid_out, hipStream_t stream) {
    int err;
    DeviceState* s = device_state(&err);
    if (!s) return err;
    int rc;
    if ((rc = ensure(s->ir_r, (size_t)n * sizeof(double)))) return rc;
    if ((rc = ensure(s->partial, (size_t)kSplits * n * sizeof(double)))) return rc;
    if ((rc = ensure(s->ir_norms, 16 * sizeof(double)))) return rc;
    // the low-precision paths' FP32 working copy, made in the same pass over A
    // as ||A||_inf
    const bool low = prec != LU_FP64;
    float* A32 = nullptr;
    if (low) {
        if ((rc = ensure(s->ir_a32, (size_t)n * n * sizeof(float)))) return rc;
        A32 = reinterpret_cast<float*>(s->ir_a32.ptr);
    }
    // ||A||_inf and a finiteness check of the inputs
    unsigned long long* nrm = reinterpret_cast<unsigned long long*>(s->ir_norms.ptr);
    if (launch_fill_zero(nrm, sizeof(unsigned long long), stream)) return LU_ERR_HIP;
    double* part = reinterpret_cast<double*>(s->partial.ptr);
    if (low ? launch_convert_row_abs_sums(A, lda, n, A32, n, part, kSplits, reinterpret_cast<double*>(nrm), stream)
            : launch_row_abs_sums(A, lda, n, part, kSplits, reinterpret_cast<double*>(nrm), stream))
        return LU_ERR_HIP;
    unsigned long long abits = 0;
    LU_HIP(hipMemcpyAsync(&abits, nrm, sizeof abits, hipMemcpyDeviceToHost, stream));
    LU_HIP(hipStreamSynchronize(stream));
    const double anorm = bits_to_double(abits);
    if (!std::isfinite(anorm)) return LU_ERR_NONFINITE;
    std::vector<double> bnorm(nrhs);
    for (int c = 0; c < nrhs; ++c) {
        if ((rc = dev_amax(s, B + (long long)c * ldb, n, stream, &bnorm[c]))) return rc;
        if (!std::isfinite(bnorm[c])) return LU_ERR_NONFINITE;
    }

    int iters_total = 0;
    double worst = 0.0;
    bool converged = true;
    // the FP64 factorization, its solve and the HPL test of every column
    auto fp64_solution = [&](bool fell_back) -> int {
        int info = 0;
        int r = fp64_path(s, n, nrhs, A, lda, B, ldb, X, ldx, stream, &info);
        if (r) return r;
        worst = 0.0;
        if (info == 0) {
            for (int c = 0; c < nrhs; ++c) {
                double res;
                if ((r = hpl_resid(s, n, A, lda, B + (long long)c * ldb, X + (long long)c * ldx, anorm, bnorm[c],
                                   stream, &res)))
                    return r;
                worst = std::isnan(res) || std::isnan(worst) ? NAN : std::max(worst, res);
            }
        }
        if (iters_out) *iters_out = iters_total;
        if (resid_out) *resid_out = info == 0 ? worst : NAN;
        return ir_outcome(info, fell_back ? 1 : 0, worst);
    };
    if (prec == LU_FP64) return fp64_solution(false);

    // low-precision factorization of the FP32 working copy
    if ((rc = ensure(s->ir_ipiv, (size_t)n * sizeof(int)))) return rc;
    if ((rc = ensure(s->ir_x32, (size_t)n * sizeof(float)))) return rc;
    int* ipiv = reinterpret_cast<int*>(s->ir_ipiv.ptr);
    float* d32 = reinterpret_cast<float*>(s->ir_x32.ptr);
    if ((rc = factor_impl(n, A32, n, prec, ipiv, nullptr, nullptr, stream))) return rc;
    int info_lp = 0;
    if ((rc = factor_status(s, stream, &info_lp))) return rc;
    if (info_lp != 0) converged = false;    // a zero pivot in the working precision: straight to FP64
    bool moves_ready = false;
    for (int c = 0; c < nrhs && converged; ++c) {
        const double* b = B + (long long)c * ldb;
        double* x = X + (long long)c * ldx;
        double* r = reinterpret_cast<double*>(s->ir_r.ptr);
        if (launch_fill_zero(x, (size_t)n * sizeof(double), stream)) return LU_ERR_HIP;
        const double bn = bnorm[c];
        double prev = INFINITY;
        int it = 0;
        for (;; ++it) {
            // x = 0 at the start: r = b needs no product, and only b = 0 passes the test
            const bool start = it == 0 && bn > 0.0;
            if (!start) {
                double res;
                if ((rc = hpl_resid(s, n, A, lda, b, x, anorm, bn, stream, &res))) return rc;   // leaves r = b - A x
                if (std::isnan(res)) { converged = false; break; }
                if (res <= 16.0) { worst = std::max(worst, res); break; }
                if (it >= max_iter || (it >= 2 && res >= prev)) { converged = false; break; }
                prev = res;
            }
            if (launch_convert_f64_f32(start ? b : r, n, d32, n, n, 1, stream)) return LU_ERR_HIP;
            if ((rc = solve_with_factor<float>(s, n, 1, A32, n, ipiv, d32, n, stream, moves_ready))) return rc;
            moves_ready = true;
            if (launch_axpy_f32_to_f64(x, d32, n, stream)) return LU_ERR_HIP;
        }
        iters_total = std::max(iters_total, it);
    }
    if ((rc = read_err(s, stream))) return rc;
    if (converged) {
        if (iters_out) *iters_out = iters_total;
        if (resid_out) *resid_out = worst;
        return LU_IR_OK;
    }
    // refinement did not reach the FP64 test: refactor in FP64
    return fp64_solution(true);
}

int solve_ex_impl(int n, int nrhs, const double* LU, int lda, const int* ipiv, double* B, int ldb,
                  hipStream_t stream) {
    int err;
    DeviceState* s = device_state(&err);
    if (!s) return err;
    return solve_with_factor<double>(s, n, nrhs, LU, lda, ipiv, B, ldb, stream, false);
}

}  // namespace lu

extern "C" {

int lu_solve_ex(int n, int nrhs, const double* LU, int lda, const int* ipiv, double* B, int ldb, hipStream_t stream) {
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (!LU && n > 0) return -3;
    if (lda < std::max(1, n)) return -4;
    if (!ipiv && n > 0) return -5;
    if (!B && n > 0 && nrhs > 0) return -6;
    if (ldb < std::max(1, n)) return -7;
    if (n == 0 || nrhs == 0) return 0;
    return lu::solve_ex_impl(n, nrhs, LU, lda, ipiv, B, ldb, stream);
}

int lu_solve(int n, int nrhs, const double* LU, const int* ipiv, double* B) {
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (!LU && n > 0) return -3;
    if (!ipiv && n > 0) return -4;
    if (!B && n > 0 && nrhs > 0) return -5;
    if (n == 0 || nrhs == 0) return 0;
    int rc = lu::solve_ex_impl(n, nrhs, LU, n, ipiv, B, n, nullptr);
    if (rc) return rc;
    int err;
    lu::DeviceState* s = lu::device_state(&err);
    if (!s) return err;
    return lu::read_err(s, nullptr);
}

int lu_ir_outcome(int fp64_info, int fell_back, double resid) { return lu::ir_outcome(fp64_info, fell_back, resid); }

int lu_solve_ir(int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X, int ldx,
                lu_precision_t prec, int max_iter, int* iters_out, double* resid_out, hipStream_t stream) {
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (!A && n > 0) return -3;
    if (lda < std::max(1, n)) return -4;
    if (!B && n > 0 && nrhs > 0) return -5;
    if (ldb < std::max(1, n)) return -6;
    if (!X && n > 0 && nrhs > 0) return -7;
    if (ldx < std::max(1, n)) return -8;
    if (prec < LU_FP64 || prec > LU_MIXED_BF16) return -9;
    if (max_iter < 1) return -10;
    if (n == 0 || nrhs == 0) {
        if (iters_out) *iters_out = 0;
        if (resid_out) *resid_out = 0.0;
        return LU_IR_OK;
    }
    return lu::solve_ir_impl(n, nrhs, A, lda, B, ldb, X, ldx, prec, max_iter, iters_out, resid_out, stream);
}

}  // extern "C"
