// Host-side launchers of the gfx950 kernels (one translation unit per kernel
// family).  All pointers are device pointers; all launches are asynchronous.
#pragma once
#include <hip/hip_runtime.h>

namespace lu {

// Composed row interchanges of one panel (see compose_moves in common.hpp):
// [0] top moves, [1] extra moves, top (dst, src) pairs from [2], extra pairs
// from [kMovesExtra]; rows relative to the panel's first row.
constexpr int kMovesMaxW = 512;
constexpr int kMovesExtra = 2 + 2 * kMovesMaxW;
constexpr int kMovesLen = 2 + 4 * kMovesMaxW;
// The panel kernel runs at most this many cooperating work-groups (rows per
// work-group <= 1024, so panels up to 65536 rows).
constexpr int kPanelMaxWgs = 64;
// size of the panel kernel's tagged exchange area, in 64-bit words (both parities)
constexpr int kPanelXchWords = 2 * (kPanelMaxWgs * (1 + 2 + 2 * 16 * 2) + 2 * 16 * 2);

template <typename T>
struct PanelArgs {
    T* A;                 // panel top-left element (panel row 0, panel column 0)
    int lda;
    int m, w;             // panel rows (from its top row to the last matrix row), width
    int row_base;         // matrix row index of panel row 0
    int* ipiv;            // ipiv[d] = row_base + pivot row, for panel columns d = 0..w-1
    int* ipiv_rel;        // optional panel-relative pivots
    int* info;            // optional LAPACK info word (first zero pivot, 1-based)
    int info_col_base;    // matrix column of panel column 0
    int* moves;           // optional composed interchanges (kMovesLen ints)
    unsigned* sync;       // [0] barrier counter (0 at launch), [1] error word
    unsigned* sync_next;  // counter of the alternate slot, zeroed by this launch
    unsigned long long* xch;   // tagged exchange area (kPanelXchWords words)
    unsigned tag_base;    // unique per launch: (launch number << 10); step d uses tag_base + d
    long long spin_limit; // barrier wait bound, wall-clock ticks
    int occupancy;        // register budget variant: 1 = whole register file, 2 = half
    int one_xcd;          // 1: all work-groups on XCD 0 (the grid holds 8 per participant)
    unsigned* rank;       // one_xcd: rank counter of the participants, 0 at launch
};

template <typename T>
int launch_panel(const PanelArgs<T>& args, int wgs, hipStream_t stream);
int panel_max_rows_per_wg();
int launch_xcd_probe(int* out, int wgs, hipStream_t stream);
int panel_threads();

template <typename T, typename H>
struct SwapTrsmArgs {
    T* A;                 // matrix base
    long long lda;
    int r0;               // first row (and column) of the panel of this step
    int w;                // panel width
    const int* moves;     // composed interchanges of the panel (rows relative to r0)
    int m;                // matrix rows from r0 on (every move row lies in [0, m))
    int c0, c1;           // columns to process
    const T* linv;        // inverses of L11's 16x16 diagonal blocks (launch_diag_inv)
    H* uh;                // optional half copy of U12: uh[col*lduh + t], t = row - r0
    long long lduh;
    float* cs;            // per-column inverse scales of uh, indexed by column
    unsigned* claim;      // non-null: XCD 0 is left free and slabs are claimed from this counter
    unsigned* claim_next; // (the counter of the next such launch on the stream, cleared by this one)
};

template <typename T, typename H>
int launch_swap_trsm(const SwapTrsmArgs<T, H>& args, hipStream_t stream);
// linv[blk*256 + k*16 + j] = inverse of the unit-lower 16x16 diagonal block
// blk of the w x w block at (r0, r0): element (j, k).  ceil(w/16) blocks.
template <typename T>
int launch_diag_inv(const T* A, long long lda, int r0, int w, T* linv, hipStream_t stream);
// rows r0 .. r0+m-1 of columns [c0, c1): the interchanges of a panel of width w
// claim non-null: XCD 0 is left free, column blocks claimed from *claim
// (claim_next: the next such launch's counter, cleared here)
template <typename T>
int launch_lswap(T* A, long long lda, int r0, int w, int m, const int* moves, int c0, int c1, hipStream_t stream,
                 unsigned* claim = nullptr, unsigned* claim_next = nullptr);
int launch_moves(const int* ipiv_rel, int w, int m, int* moves, hipStream_t stream);
// Deferred left interchanges (update.hip, lperm_kernel): every panel k < N-1
// of the factorization takes the interchanges of all later panels; moves of
// panel j at moves + j*kMovesLen; starts on the host and on the device
// (N+1 ints).  Needs n - starts[1] <= kLpermMaxRows.
constexpr int kLpermThreads = 1024;
constexpr int kLpermCols = 32;          // columns per work-group
constexpr int kLpermMaxRows = 32768;    // rows of a column segment (32 per thread; the LDS holds one int per row)
template <typename T>
int launch_lperm(T* A, long long lda, int n, int N, const int* starts_host, const int* starts_dev, const int* moves,
                 hipStream_t stream);
int launch_chunk_moves(const int* ipiv, int n, int W, int* moves, hipStream_t stream);
template <typename H>
int launch_l21_half(const float* A, long long lda, int m, int w, H* Lh, long long ldh, float* rs,
                    hipStream_t stream);

template <typename H>
int launch_cols_half(const float* B, long long ldb, int k, int n, H* Uh, long long ldh, float* cs,
                     hipStream_t stream);

// Counters of a launch that leaves XCD 0 free for a panel running there: the
// work-groups on XCD 0 return at once, the others claim tiles from per-XCD
// chunks (8 counters, `next` = those of the next such launch on the stream,
// cleared by this one); `cus` sizes the persistent grid.
struct XcdClaim {
    unsigned* ctr = nullptr;
    unsigned* next = nullptr;
    int cus = 0;
};
// claim.ctr null: one work-group per tile on every XCD.
template <typename T>
int launch_gemm(int M, int N, int K, const T* A, int lda, const T* B, int ldb, T* C, int ldc, hipStream_t stream,
                XcdClaim claim = XcdClaim());
// C -= A B for the Householder block updates (the trailing-update tile, its own kernel name)
template <typename T>
int launch_gemm_hh(int M, int N, int K, const T* A, int lda, const T* B, int ldb, T* C, int ldc, hipStream_t stream);
// slices z of ks k-values: C + z*cstride = -A[:, slice] B[slice, :] (not accumulated)
template <typename T>
int launch_gemm_split(int M, int N, int K, int ks, const T* A, int lda, const T* B, int ldb, T* C, int ldc,
                      long long cstride, hipStream_t stream);
template <typename H>
int launch_gemm_half(int M, int N, int K, const H* Ah, int lda_h, const H* Bh, int ldb_h, const float* rs,
                     const float* cs, float* C, int ldc, hipStream_t stream, XcdClaim claim = XcdClaim());
int launch_probe_mfma_f64(double* out, hipStream_t stream);

// Symmetric update C -= A B^T on C's lower triangle (element (i,j) when
// i + diag >= j); B is given transposed, element (k, j) at B[j + k*ldb].
template <typename T>
int launch_syrk_lower(int M, int N, int K, const T* A, int lda, const T* B, int ldb, T* C, int ldc, int diag,
                      hipStream_t stream);

// Cholesky panel (chol.hip): the m x w column block at A (its diagonal at
// A[0]), lower triangle, w <= 512; persistent multi-work-group launch.
template <typename T>
struct CholPanelArgs {
    T* A;
    long long lda;
    int m, w;
    int* info;             // device; first non-positive pivot (1-based), set once
    int info_col_base;     // global column of the panel's first column
    unsigned* sync;        // [counter, error] of this launch's barrier
    unsigned* sync_next;   // counter the next launch will use (cleared here)
    long long spin_limit;  // wall-clock ticks a barrier may wait
};
template <typename T>
int launch_chol_panel(const CholPanelArgs<T>& args, int wgs, hipStream_t stream);

// Householder QR panel (qr.hip): the m x w column block at A (its diagonal at
// A[0]), FP64, w <= 256, m <= 1024 * wgs; persistent multi-work-group launch.
struct QrPanelArgs {
    double* A;
    long long lda;
    int m, w;
    double* tau;           // w reflector scalars (device)
    double* T;             // w x w upper triangular block-reflector factor, ld w (device)
    double* part;          // kQrPartWords doubles of partial sums (device)
    unsigned* sync;        // [counter, error] of this launch's barrier
    unsigned* sync_next;   // counter the next launch will use (cleared here)
    long long spin_limit;
};
// workspace of the QR panel: per-group partial sums and the block-phase W
constexpr int kQrMaxPanelW = 384;
constexpr int kQrPanelGroupRows = 1024;  // panel rows per work-group (the launch has ceil(m / 1024) groups)
constexpr int kQrPanelMaxGroups = 64;
constexpr int kQrPartWords = 2 * kQrPanelMaxGroups + kQrPanelMaxGroups * 16 + kQrPanelMaxGroups * 16 * kQrMaxPanelW +
                             16 * kQrMaxPanelW;
int launch_qr_panel(const QrPanelArgs& args, int wgs, hipStream_t stream);
// Vw (m x w, ld m) and VT (w x m, ld w): the panel's unit-lower V, explicit;
// TT = T^T (w x w, ld w)
int launch_qr_prep(const double* A, long long lda, int m, int w, const double* T, double* Vw, double* VT,
                   double* TT, hipStream_t stream);
// W = sum of the S k-slices Wp[s * count ...] in slice order
int launch_qr_wsum(const double* Wp, int S, long long count, double* W, hipStream_t stream);
// dst (cols x rows, ld ldd) = src^T, src rows x cols with ld lds
int launch_transpose_f64(const double* src, long long lds, int rows, int cols, double* dst, long long ldd,
                         hipStream_t stream);

// ---- solves and refinement (solve.hip) ----
// x (n x nrhs, ld) <- P x using per-chunk moves from launch_chunk_moves
template <typename T>
int launch_apply_chunk_moves(T* X, long long ldx, int n, int nrhs, int W, const int* moves, hipStream_t stream);
// triangular solves with the packed LU factor; flags: int[nblocks] epoch flags
template <typename T>
int launch_trsv_lower_unit(const T* LU, long long lda, int n, T* x, int* flags, int epoch, unsigned* err,
                           long long spin_limit, hipStream_t stream);
// Cholesky solve of one right-hand side in place: L y = x, then L^T x = y
// (L lower with its diagonal, column-major); one flag epoch per triangle.
template <typename T>
int launch_trsv_chol(const T* L, long long lda, int n, T* x, int* flags, int epoch_lower, int epoch_upper,
                     unsigned* err, long long spin_limit, hipStream_t stream);
template <typename T>
int launch_trsv_upper(const T* LU, long long lda, int n, T* x, int* flags, int epoch, unsigned* err,
                      long long spin_limit, hipStream_t stream);
constexpr int kTrsvRows = 64;     // rows per block of the blocked triangular solves (one ready flag each)
int trsv_block_rows();

// IR building blocks (FP64 residual side)
int launch_residual(const double* A, long long lda, int n, const double* x, const double* b, double* r,
                    double* partial, int splits, hipStream_t stream);
int launch_row_abs_sums(const double* A, long long lda, int n, double* partial, int splits, double* out_max,
                        hipStream_t stream);
int launch_amax(const double* x, int n, unsigned long long* out_bits, hipStream_t stream);
int launch_convert_f64_f32(const double* src, long long lds, float* dst, long long ldd, int rows, int cols,
                           hipStream_t stream);
int launch_axpy_f32_to_f64(double* x, const float* d, int n, hipStream_t stream);
int launch_copy_f64(const double* src, long long lds, double* dst, long long ldd, int rows, int cols,
                    hipStream_t stream);
int launch_fill_zero(void* p, size_t bytes, hipStream_t stream);

// selector network (mlp.hip)
int launch_mlp_forward(const float* theta, const float* X, int batch, float* logits, hipStream_t stream);
int launch_mlp_train(float* theta, float* m, float* v, const float* X, const int* Y, int batch, int epochs,
                     float lr, int t0, float* loss_out, float* grad_out, int update, hipStream_t stream);

}  // namespace lu
