/*
 * lu.h -- C ABI of the MI355X (gfx950) look-ahead LU library.
 *
 * Method: blocked right-looking LU factorization with partial pivoting,
 * P*A = L*U, in which the factorization of the next panel overlaps the
 * trailing update of the current one (static look-ahead).  The operations
 * per step k follow the paper:
 *   Sec. 3.5, LU_blk:  RL1 [A11;A21] := LU_unb([A11;A21])      (panel)
 *                      RL2 A12 := trilu(A11)^-1 A12              (TRSM)
 *                      RL3 A22 := A22 - A21 A12                  (GEMM)
 *   Sec. 3.4: LAPACK getrf = getf2 -> laswp -> trsm -> gemm; the row
 *             interchanges of the panel are applied to the columns on both
 *             sides of it (laswp);
 *   Sec. 4 (Listing 5): TU_k splits into TU_k^L (the columns of panel k+1)
 *             and TU_k^R (the rest); PU(k+1) = TU_k^L + PF(k+1) runs
 *             concurrently with TU_k^R;
 *   Sec. 4.2: when the panel work ends early its resources rejoin the
 *             trailing update.
 * The look-ahead reorders operations only: the factors equal those of plain
 * Gaussian elimination with partial pivoting up to floating-point rounding.
 *
 * Conventions for every entry point
 *   - Matrices are column-major: element (i,j) at ptr[i + j*ld], ld >= max(1,n).
 *   - Matrix, vector and pivot pointers are DEVICE pointers owned by the
 *     caller, unless a parameter says "host".  The library never frees them.
 *   - ipiv is int32[n], 0-based, LAPACK semantics: at step k rows k and
 *     ipiv[k] (>= k) were interchanged.
 *   - Return 0 on success; -i if argument i (1-based) is illegal, checked
 *     before any GPU call; LU_ERR_* (<= -100) for runtime failures.
 *   - n == 0 returns 0 without touching the GPU.
 *   - A singular U is not an error: the factorization completes and info
 *     reports the first exactly-zero pivot (1-based column), as LAPACK does.
 *   - Calls are asynchronous on `stream` unless stated otherwise, and are not
 *     thread-safe: one host thread per device at a time.  The factorizations
 *     run on the library's own update and panel streams (created together so
 *     that they use different hardware queues), ordered after `stream` on
 *     entry; `stream` waits for them on exit (events), so work enqueued on it
 *     afterwards sees the result.
 *   - The library owns its workspace (device buffers, its streams, events),
 *     cached per device until lu_release().
 */
#ifndef LU_MI355X_H
#define LU_MI355X_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LU_FP64 = 0,        /* FP64 throughout (MFMA f64 trailing update)                 */
    LU_FP32 = 1,        /* FP32 storage, panel, TRSM and GEMM                         */
    LU_MIXED_FP16 = 2,  /* FP32 storage/panel/TRSM; trailing GEMM on FP16 operands,
                           FP32 accumulation; per-row/per-column power-of-two scales  */
    LU_MIXED_BF16 = 3   /* as LU_MIXED_FP16 with BF16 operands                        */
} lu_precision_t;

/* Schedule: algorithmic block size b, look-ahead depth (0 = none, the
 * conventional loop; 1 = the paper's one-panel look-ahead; 2 = two panels),
 * the number of compute units given to the panel work, and the panel taper
 * (early termination done statically, Sec. 4.2: 1 = panels narrow to 128
 * columns once the trailing matrix is small, see lu_plan_panels in
 * lu_plan.h; -1 = every panel b wide).  A field 0 (b, panel_cus, taper) or
 * < 0 (b, depth, panel_cus) means "choose" (explicit value > environment >
 * selector > default; the taper's default is on). */
typedef struct {
    int b;
    int depth;
    int panel_cus;
    int taper;
} lu_schedule_t;

#define LU_ERR_HIP         (-100)  /* a HIP runtime call failed                           */
#define LU_ERR_BARRIER     (-101)  /* a device-wide panel barrier timed out               */
#define LU_ERR_NOMEM       (-102)  /* workspace allocation failed                         */
#define LU_ERR_UNSUPPORTED (-103)  /* size or option outside what the library supports  */
#define LU_ERR_NONFINITE   (-104)  /* NaN/Inf met where a finite value is required        */
#define LU_ERR_SINGULAR    (-105)  /* lu_solve_ir: the FP64 factor has an exactly-zero pivot */

#define LU_IR_OK         0  /* the solution meets the FP64 HPL residual test (<= 16)        */
#define LU_IR_FELL_BACK  1  /* refinement stalled or the working-precision factor was
                               singular; the FP64 factorization was used and its solution
                               meets the test                                             */
#define LU_IR_RESID_HIGH 2  /* the FP64 solution (LU_FP64, or after the fall-back) fails
                               the HPL test; X holds it                                   */

/* ---- factorization ----------------------------------------------------- */

/* Factor the n x n FP64 matrix A in place (L below the diagonal with an
 * implicit unit diagonal, U on and above it) and write the pivots to ipiv.
 * Uses the default/selected schedule.  Enqueued on `stream`; returns without
 * a host synchronisation.  Errors: -1 n<0, -2 A==NULL, -3 lda<max(1,n),
 * -4 ipiv==NULL. */
int lu_factor(int n, double* A, int lda, int* ipiv, hipStream_t stream);

/* General form.  A is double* for LU_FP64 and float* for the other three
 * precisions.  sched may be NULL (all fields "choose").  d_info, if not NULL,
 * is a device int that receives LAPACK INFO (0, or the 1-based index of the
 * first zero pivot); it must be zeroed by the caller before the call.
 * Errors as lu_factor, plus -5 unknown precision, -6 illegal schedule field
 * (b not in {32,64,128,256,512}, depth not in {0,1,2}, panel_cus > 256). */
int lu_factor_ex(int n, void* A, int lda, lu_precision_t prec, int* ipiv,
                 const lu_schedule_t* sched, int* d_info, hipStream_t stream);

/* Synchronise with the stream of the most recent factorization on the
 * current device and return its INFO through *info (host pointer).  Returns
 * LU_ERR_BARRIER if a panel barrier timed out in that factorization. */
int lu_factor_info(int* info);

/* The schedule the library would use for (n, prec) with no explicit fields
 * (environment LU_B / LU_DEPTH / LU_PANEL_CUS, then the selector, then the
 * default b=256, depth=1, panel_cus=16).  out is a host pointer. */
int lu_schedule_default(int n, lu_precision_t prec, lu_schedule_t* out);

/* ---- solves --------------------------------------------------------------- */

/* Solve A X = B with the factors of lu_factor (LAPACK getrs, no transpose):
 * B <- U^-1 L^-1 P B.  Square leading dimensions lda = ldb = n; null stream;
 * returns after the solve completes.  Errors: -1 n<0, -2 nrhs<0, -3 LU==NULL,
 * -4 ipiv==NULL, -5 B==NULL. */
int lu_solve(int n, int nrhs, const double* LU, const int* ipiv, double* B);

/* General form of lu_solve, asynchronous on `stream`.  Errors: -1 n, -2 nrhs,
 * -3 LU, -4 lda, -5 ipiv, -6 B, -7 ldb. */
int lu_solve_ex(int n, int nrhs, const double* LU, int lda, const int* ipiv,
                double* B, int ldb, hipStream_t stream);

/* lu_solve_ex for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and result, with the scratch memory (interchange lists,
 * ready flags, error word; 1 053 952 bytes) in one statically allocated device
 * array per GPU instead of library-allocated buffers.  Calls no hipMalloc,
 * hipFree or other allocating routine and creates no stream or event; the
 * array's address is looked up once per device, on the first call with that
 * device current.  Every call on one GPU shares its array: calls on that GPU
 * that overlap in time (on different streams, or from several host threads)
 * race and must be serialised by the caller.  Arguments, errors and stream
 * semantics as lu_solve_ex, plus LU_ERR_UNSUPPORTED when n > LU_NOALLOC_MAX_N.
 * As with lu_solve_ex, a wait of the triangular solves that times out is not
 * reported. */
#define LU_NOALLOC_MAX_N 65536
int lu_solve_noalloc(int n, int nrhs, const double* LU, int lda, const int* ipiv,
                     double* B, int ldb, hipStream_t stream);

/* Mixed-precision solve with FP64 iterative refinement (not in the paper;
 * the precision axis of this library).  A (FP64) and B are read, never
 * written; X receives the solution.  The LU of a working copy of A is
 * computed in `prec` (LU_FP32 / LU_MIXED_FP16 / LU_MIXED_BF16; LU_FP64 gives
 * plain FP64 LU + solve + the same residual test), then
 *     r = B - A X (FP64),  solve (L U) d = P r in the working precision,
 *     X += d (FP64)
 * repeats until every column meets the HPL test
 *     ||A x - b||_inf / (eps (||A||_inf ||x||_inf + ||b||_inf) n) <= 16,
 *     eps = 2^-53,
 * or max_iter iterations pass.  Without convergence (or when the working-
 * precision factor has a zero pivot) the matrix is refactored in FP64 and
 * solved plainly.  Synchronises the stream (the convergence test is read on
 * the host each iteration).  The INFO word and the panel barriers of every
 * factorization it runs are checked.
 * iters_out / resid_out (host, may be NULL) receive the refinement steps taken
 * and the final worst-column HPL residual (NaN when no FP64 solution exists).
 * Returns LU_IR_OK, LU_IR_FELL_BACK, LU_IR_RESID_HIGH (the FP64 solution
 * fails the test), LU_ERR_SINGULAR (the FP64 factor has a zero pivot; X is
 * not written), LU_ERR_NONFINITE (NaN/Inf in A or B, or in the residual),
 * LU_ERR_BARRIER (a panel barrier timed out), or an argument error: -1 n,
 * -2 nrhs, -3 A, -4 lda, -5 B, -6 ldb, -7 X, -8 ldx, -9 prec,
 * -10 max_iter < 1. */
int lu_solve_ir(int n, int nrhs, const double* A, int lda, const double* B, int ldb,
                double* X, int ldx, lu_precision_t prec, int max_iter,
                int* iters_out, double* resid_out, hipStream_t stream);

/* ---- learned schedule selector ---------------------------------------------
 * A 4 -> 32 -> 10 perceptron (inputs: log2 n scaled, precision one-hot of
 * FP64 / FP32 / mixed-FP16; heads: b in {64,128,256,512}, depth in {0,1,2},
 * panel_cus in {8,16,32}).  Inference and training run in the library's own
 * GPU kernels. */

/* Load weights written by lu_selector_save / the training script (host path).
 * Returns 0, or <0 if the file is missing or corrupt, in which case whatever
 * was active before (weights, or the fixed default) stays active.
 * path == NULL drops the active weights: the fixed default is used from then
 * on, also for the weights file next to the library (returns 0). */
int lu_selector_load(const char* path);

/* Predict the schedule for (n, prec) into *out (host).  Returns 0, or 1 when
 * no weights are loaded or n lies outside [0.5x, 2x] of the training range,
 * in which case *out holds the fixed default. */
int lu_selector_predict(int n, lu_precision_t prec, lu_schedule_t* out);

/* Train the network on the GPU: X is host float[batch*4], Y host int[batch*3]
 * (class index per head), `epochs` full-batch Adam steps with learning rate
 * lr, from the current weights (or a seeded initialisation when none are
 * loaded and `seed` >= 0).  loss_out (host, may be NULL) receives the loss
 * after every epoch (float[epochs]).  The trained weights become active. */
int lu_selector_train(const float* X, const int* Y, int batch, int epochs, float lr,
                      int seed, float* loss_out);

/* Save / read the active weights (host float[490], order W1 32x4 row-major,
 * b1[32], W2 10x32 row-major, b2[10]) plus the feature range. */
int lu_selector_save(const char* path);
int lu_selector_get_params(float* theta_out, int n_theta);
int lu_selector_set_params(const float* theta, int n_theta, int n_min, int n_max);

/* One forward+backward pass on the GPU without updating: loss and gradient
 * (host float[490]) of the current weights on a batch. */
int lu_selector_grad(const float* X, const int* Y, int batch, float* loss_out,
                     float* grad_out);

/* Free every library-owned resource on every device used so far. */
void lu_release(void);

#ifdef __cplusplus
}
#endif

#endif /* LU_MI355X_H */
