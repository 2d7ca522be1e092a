/*
 * lu_plan.h -- the look-ahead schedule as an inspectable task list.
 *
 * The factorization is a DAG over elimination steps k = 0..N-1 on panels
 * [s_j, s_j+1) (s_0 = 0, s_N = n).  With a fixed block size b, s_j = jb
 * (N = ceil(n/b); the last panel has width n-(N-1)b when b does not divide
 * n); with the early-termination taper (Sec. 4.2) the panels narrow as the
 * trailing matrix shrinks (lu_plan_panels):
 *   PANEL(j)        factor panel j: columns [s_j, s_j+1), rows >= s_j
 *                   (RL1 of LU_blk, Sec. 3.5), producing ipiv[jb..jb+w_j)
 *   UPDATE(k,c0,c1) apply step k to columns [c0,c1): the interchanges of
 *                   panel k, RL2 (U12 := trilu(A11)^-1 A12) and RL3
 *                   (A22 -= A21 A12) (Sec. 3.4, 3.5)
 *   LSWAP(k,0,s_k)  apply the interchanges of panel k to the finished
 *                   columns left of it (the left half of laswp, Sec. 3.4)
 *   LPERM(N-1,0,s_N-1) the same for every panel at once, deferred to the end:
 *                   the columns of each panel k take the interchanges of all
 *                   later panels (rows >= s_k+1) in one permutation per
 *                   column.  Nothing reads those columns again before the
 *                   end, so the result equals that of the LSWAP tasks.
 * A schedule places these tasks in a program order that is a valid
 * sequential order of the algorithm (Listing 3 for depth 0, Listing 5 of
 * Sec. 4 for depth 1, two panels ahead for depth 2) and assigns each to one
 * of LU_PLAN_STREAMS streams: 0 = the update stream (the caller's stream),
 * 1 = the panel stream, 2 = the stream of the left interchanges (depth >= 1;
 * depth 0 keeps every task on stream 0).  Each task lists the earlier tasks
 * of OTHER streams it must wait for (at most one per stream); these are
 * derived mechanically from the column ranges and pivot
 * blocks each task reads and writes, so concurrently runnable tasks touch
 * disjoint data and every execution order the streams allow gives the
 * result of the program order.
 */
#ifndef LU_MI355X_PLAN_H
#define LU_MI355X_PLAN_H

#ifdef __cplusplus
extern "C" {
#endif

#define LU_TASK_PANEL  0
#define LU_TASK_UPDATE 1
#define LU_TASK_LSWAP  2
#define LU_TASK_LPERM  3

#define LU_PLAN_STREAMS  3
#define LU_PLAN_MAX_WAIT 2   /* = LU_PLAN_STREAMS - 1 */

typedef struct {
    int kind;                   /* LU_TASK_*                                          */
    int step;                   /* k (PANEL: the panel index j)                       */
    int col_begin, col_end;     /* columns written, [col_begin, col_end)              */
    int stream;                 /* 0 update, 1 panel, 2 left interchanges             */
    int nwait;                  /* cross-stream waits                                 */
    int wait[LU_PLAN_MAX_WAIT]; /* indices of earlier tasks (other streams) to wait on */
    int record;                 /* 1 if a later task waits on this one                */
} lu_plan_task_t;

/* Build the task list for an n x n factorization with block size b and
 * look-ahead depth (0, 1 or 2) into out[0..max_tasks) (host memory).
 * Pure host code: no GPU call.  Returns the number of tasks, or -1 n<0,
 * -2 b<1, -3 depth not in {0,1,2}, -5 max_tasks too small (the return value
 * is then -5 and nothing beyond max_tasks is written). */
int lu_plan_build(int n, int b, int depth, lu_plan_task_t* out, int max_tasks);

/* Panel boundaries of a schedule, into starts[0..N] (host memory; starts[0] = 0,
 * starts[N] = n); returns N.  taper <= 0: every panel b wide (the last one
 * ragged).  taper > 0: early termination done statically (Sec. 4.2) -- the
 * panel starting at column s is min(b, t) wide, where t depends on the trailing
 * size n - s and the precision class prec (lu_precision_t: 0 FP64, 1 FP32,
 * 2/3 mixed): t = 128 for n - s <= 12288 (FP64) or <= 16384 (FP32, mixed),
 * unbounded beyond.
 * Pure host code.  Returns -1 n<0, -2 b<1, -4 prec out of range, -5 starts
 * NULL or max_starts < N+1 (nothing written); 0 for n = 0. */
int lu_plan_panels(int n, int b, int taper, int prec, int* starts, int max_starts);

/* The task list for explicit panel boundaries starts[0..npanels] (host memory,
 * strictly increasing from 0 to n, e.g. from lu_plan_panels), as
 * lu_plan_build.  Returns the number of tasks, or -1 n<0, -3 depth not in
 * {0,1,2}, -4 invalid boundaries, -5 max_tasks too small. */
int lu_plan_build_panels(int n, const int* starts, int npanels, int depth, lu_plan_task_t* out,
                         int max_tasks);

/* As lu_plan_build_panels; interchanges = 0 gives the task list of the
 * factorizations without row interchanges (Cholesky, QR: no LU_TASK_LSWAP
 * tasks and no waits on pivots), 1 the LU's with one LU_TASK_LSWAP per
 * step (as lu_plan_build_panels), 2 the LU's with the left interchanges
 * deferred to one final LU_TASK_LPERM task (on stream 0).  Same returns, and
 * -6 for another value of interchanges. */
int lu_plan_build_panels_ex(int n, const int* starts, int npanels, int depth, int interchanges,
                            lu_plan_task_t* out, int max_tasks);

#ifdef __cplusplus
}
#endif

#endif /* LU_MI355X_PLAN_H */
