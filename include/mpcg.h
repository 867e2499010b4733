/*
 * mpcg.h -- C ABI of the MI355X (gfx950) restarted mixed-precision CG library.
 *
 * The method (Prolubnikov, "Parameter Optimization for Restarted
 * Mixed-Precision Iterative Sparse Solver", arXiv 2412.08059):
 *   Algorithm I  -- CG on float32(A), float32(b) from x~0 = 0 down to the
 *                   tolerance eps1, then float64(x~) as the start of FP64 CG on
 *                   A x = b down to eps2 (sections "Two-Stage Algorithm ..."
 *                   and "Conjugate Gradient Method").
 *   Algorithm II -- the same, with eps1 picked per matrix: k0 FP32 iterations
 *                   give v, the mean of ||r_i|| / ||r_{i-1}|| (eq. 13); the
 *                   feature vector chi = (n, m, pseudo-diameter, v) is
 *                   classified by weighted kNN into eps1 = 10^-t, t = 2..7
 *                   (eq. 23), and the FP32 recurrence continues from iterate
 *                   k0 (Remark 3).
 *   2BFS         -- pseudo-diameter of the matrix graph by two breadth-first
 *                   sweeps, maximised over connected components (section
 *                   "Computing Pseudo-Diameter of the Graph Matrix").
 *
 * Conventions for every entry point:
 *   - Every call returns an mpcg_status; 0 is success, negatives are errors.
 *     No C++ exception crosses the ABI.
 *   - Matrix, vector and output pointers are DEVICE pointers (hipMalloc or
 *     torch tensors on the same GPU) unless stated otherwise; struct
 *     arguments (mpcg_csr, mpcg_stats, mpcg_features_t, mpcg_options) are
 *     HOST memory.
 *   - The caller owns every buffer.  The library allocates no device memory:
 *     all scratch lives in the arena handed over by mpcg_set_workspace.  It
 *     allocates a few KB of pinned host memory per context for the readbacks,
 *     and captures HIP graphs (whose memory the HIP runtime owns) for the
 *     batched engine's steps and the rounds of the bit-parallel 2BFS.
 *   - All work is enqueued on the context's stream; a call returns after its
 *     results are complete (it synchronises that stream).  One context per
 *     host thread and stream; calls on one context must not overlap.
 *   - Tolerances are relative to ||b||_2 (tol_mode 0) or absolute (tol_mode 1).
 */
#ifndef MPCG_H
#define MPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPCG_OK = 0,
    MPCG_EINVAL = -1,     /* bad argument or malformed CSR; nothing was written */
    MPCG_ENOTSPD = -2,    /* d^T A d <= 0 in the FP64 phase */
    MPCG_ENOCONV = -3,    /* FP64 iteration cap or restart cap reached; x holds the last iterate */
    MPCG_ENOMEM = -4,     /* workspace missing or smaller than mpcg_workspace_size */
    MPCG_EDEVICE = -5,    /* a HIP runtime call failed or a device-side guard tripped */
    MPCG_ENONFINITE = -6, /* NaN/Inf in A or b, or a non-finite d^T A d in the FP64 phase */
    MPCG_EBUSY = -7,      /* batch engine full */
    MPCG_ECANCELED = -8,  /* batch request cancelled */
    MPCG_ENOMODEL = -9    /* eps1 = MPCG_EPS1_AUTO without a loaded kNN model */
} mpcg_status;

/* CSR matrix A (n x n), 0-based, DEVICE arrays.
 *   row_ptr  n+1 entries, int32 (row_ptr_is_i64 = 0) or int64 (= 1);
 *            row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz < 2^31.
 *   col_idx  nnz int32 column indices, strictly increasing within a row.
 *   val      nnz float64 values, finite, no stored zeros.
 * The pattern is expected to be symmetric (A is SPD); it is not checked.
 * The 2BFS takes the pattern as an undirected graph (its narrow-band levels
 * find a row's neighbours from the rows that list it), so with an
 * unsymmetric pattern the features are unspecified. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const void *row_ptr;
    int32_t row_ptr_is_i64;
    int32_t pad_;
    const int32_t *col_idx;
    const double *val;
} mpcg_csr;

/* chi(A) = (n, m, pseudo-diameter, v) and the 2BFS by-products. */
typedef struct {
    int64_t n;            /* rows */
    int64_t m;            /* stored entries (nnz, diagonal included) */
    int64_t pdiam;        /* 2BFS pseudo-diameter, max over components */
    int64_t bfs_t;        /* farthest vertex of the first sweep (component attaining pdiam) */
    int64_t bfs_u;        /* farthest vertex of the second sweep */
    int32_t n_components; /* connected components of the matrix graph */
    int32_t k0_used;      /* FP32 iterations that entered v (< k0 only if CG ended early) */
    double v;             /* eq. (13) */
} mpcg_features_t;

#define MPCG_FLAG_FP32_BREAKDOWN 1   /* FP32 d^T A d <= 0 or non-finite: switched to FP64 early */
#define MPCG_FLAG_FP32_MAXIT 2       /* FP32 phase hit maxit1: switched to FP64 */
#define MPCG_FLAG_FINAL_RESTARTED 4  /* final true residual above eps2: FP64 restarted from b - Ax */
#define MPCG_FLAG_KNN_EXACT 8        /* a training sample had zero distance to chi */
#define MPCG_FLAG_BFS_DIA 16         /* the 2BFS ran as bit-parallel levels over the diagonals
                                        (mpcg_tuning.bfs_dia); the features are the same integers */

typedef struct {
    int32_t n1;           /* FP32 iterations (the k0 prefix included) */
    int32_t n2;           /* FP64 iterations */
    int32_t restarts;     /* FP64 restarts after the final check */
    int32_t flags;        /* MPCG_FLAG_* */
    int32_t eps1_class;   /* t of eps1 = 10^-t chosen by kNN, -1 otherwise */
    int32_t status;       /* same as the return value */
    double eps1_used;     /* eps1 of the FP32 phase (-1 for FP64-only) */
    double relres_sp;     /* recursive ||r~|| / ||b|| when the FP32 phase stopped */
    double relres_restart_true; /* ||b - A float64(x~)|| / ||b|| at the restart */
    double relres_final_true;   /* ||b - A x|| / ||b|| of the returned x */
    double omega_measured;      /* (t_sp / n1) / (t_dp / n2), 0 if undefined */
    double I_third;             /* n1 / 3 + n2, eq. (4) with omega = 1/3 */
    double I_meas;              /* omega_measured * n1 + n2 */
    double t_feat_ms;           /* 2BFS (Algorithm II only; runs beside the FP32 phase) */
    double t_sp_ms;             /* call start to the FP64 restart: ingest, FP32 phase, kNN */
    double t_dp_ms;             /* restart + FP64 phase + final check(s) */
    double t_total_ms;
    mpcg_features_t feat;       /* filled for eps1 = MPCG_EPS1_AUTO */
} mpcg_stats;

typedef struct {
    int32_t k0;           /* FP32 iterations for v (Algorithm II); default 20, at most 64 */
    int32_t knn_k;        /* neighbours; 0 = the model's k */
    int32_t tol_mode;     /* 0 relative to ||b|| (default), 1 absolute */
    int32_t max_restarts; /* FP64 restarts after a failed final check; default 5 */
    int32_t graph_iters;  /* CG iterations enqueued between host polls; 0 = default (8) */
    int32_t precond;      /* 0 none (default); 1 Jacobi, M = diag(A), in both stages (the
                             preconditioned CG procedure of the subsection "Propagation of
                             Rounding Errors When Precondition is Applied"): a row without a
                             positive finite diagonal entry makes mpcg_solve return ENOTSPD;
                             not available to the batch engine */
    int64_t maxit1;       /* FP32 cap; <= 0: n */
    int64_t maxit2;       /* FP64 cap; <= 0: max(10 n, 1000) */
    int32_t dot_acc;      /* FP32-phase dot products (d.q, r.r, r.z): 0 accumulate in FP64
                             (default; each FP32 x FP32 product is exact there), 1 accumulate in
                             FP32 -- the paper leaves the accumulation precision of the FP32 phase
                             open (Remark 3 only fixes the FP64 norms of v) */
    int32_t spmv_variant; /* sparse product: 0 auto (the loaded tuning table, else SELL-64 when
                             its padding fits, split in two launches for 32-bit columns);
                             1 SELL-64 fused; 2 SELL-64 split (direction, then a one-vector
                             gather); 3 CSR stream.  Every variant runs each row's fma chain in
                             CSR order, so the products are the same bits */
    int32_t bfs_mode;     /* 2BFS large levels: 0 auto (tuning table, else one launch per
                             level); 1 one launch per level; 2 one persistent launch with a grid
                             barrier (falls back to 1 if its blocks cannot all be resident) */
    int32_t pad_;
} mpcg_options;

typedef struct mpcg_ctx mpcg_ctx;

#define MPCG_EPS1_AUTO 0.0     /* Algorithm II: features + kNN choose eps1 */
#define MPCG_EPS1_NONE (-1.0)  /* FP64-only CG from x0 = 0 (the comparator) */

/* Create a context bound to the current HIP device and to hip_stream
 * (a hipStream_t; NULL = the default stream).  opt may be NULL (defaults).
 * Errors: EINVAL (ctx NULL or options out of range), EDEVICE. */
mpcg_status mpcg_create(mpcg_ctx **ctx, const mpcg_options *opt, void *hip_stream);

/* Release the context and its pinned host buffers (not the workspace). */
mpcg_status mpcg_destroy(mpcg_ctx *ctx);

/* Bytes of device workspace needed for systems up to n rows and nnz entries. */
mpcg_status mpcg_workspace_size(const mpcg_ctx *ctx, int64_t n, int64_t nnz, size_t *bytes);

/* Hand the library a device arena (>= mpcg_workspace_size, 256-byte aligned).
 * The caller keeps ownership and must keep it alive while the context uses it. */
mpcg_status mpcg_set_workspace(mpcg_ctx *ctx, void *dev_arena, size_t bytes);

/* Load the kNN model file (host path).  Text format: header lines
 * "mpcg-knn-model 1", "k K", "mask M", "omega W", "ns N", "fmin f0..f3",
 * "fmax f0..f3", then N lines "n m ell v t".  EINVAL on a malformed file. */
mpcg_status mpcg_load_model(mpcg_ctx *ctx, const char *path);

/* Algorithm II features of A: n, m, 2BFS pseudo-diameter (per component,
 * maximised) and v over the first k0 FP32 CG iterations on float32(A) x =
 * float32(b) from 0.  b is a device float64[n]. */
mpcg_status mpcg_features(mpcg_ctx *ctx, const mpcg_csr *A, const double *b, int32_t k0,
                          mpcg_features_t *out);

/* Weighted kNN on host features: min-max normalisation from the model,
 * squared Euclidean search, 1/rho weights (eq. 23); ties to the larger eps1.
 * Writes eps1 = 10^-t and t.  ENOMODEL without a model. */
mpcg_status mpcg_select_eps1(const mpcg_ctx *ctx, const mpcg_features_t *f, double *eps1,
                             int32_t *cls);

/* Solve A x = b.  x is a device float64[n] output (its input value is ignored;
 * x0 = 0).  eps1 > 0: Algorithm I with that eps1; MPCG_EPS1_AUTO: Algorithm II;
 * MPCG_EPS1_NONE: FP64-only CG.  eps2 > 0 is the final tolerance, checked on
 * the true residual b - A x.  stats may be NULL.
 * ||b|| = 0 returns x = 0 and MPCG_OK. */
mpcg_status mpcg_solve(mpcg_ctx *ctx, const mpcg_csr *A, const double *b, double *x, double eps1,
                       double eps2, mpcg_stats *stats);

/* mpcg_solve for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same solve, with
 * the workspace taken from a device array built into the library (160 MiB on
 * every GPU the library runs on, held until the process ends) instead of the
 * context's arena, so it needs no mpcg_set_workspace and calls no hipMalloc,
 * hipFree or other allocating routine, and captures no graphs (its 2BFS rounds
 * are plain launches).  Algorithm II (eps1 = MPCG_EPS1_AUTO) still starts one
 * host thread for its 2BFS, as mpcg_solve does.
 * Arguments, results and errors are those of mpcg_solve, plus ENOMEM when the
 * system's workspace (mpcg_workspace_size for its n and nnz) exceeds the
 * array -- about 4e5 rows of a 7-point stencil fit.  Every call on a GPU
 * uses that GPU's one array: calls that overlap on one GPU (other contexts,
 * other threads) race and must be serialised by the caller. */
mpcg_status mpcg_solve_noalloc(mpcg_ctx *ctx, const mpcg_csr *A, const double *b, double *x, double eps1,
                               double eps2, mpcg_stats *stats);

/* y = A x with the solver's SpMV kernel (one fma chain per row in CSR order).
 * precision 64: x, y float64; precision 32: x, y float32 and A rounded to
 * float32 (round to nearest even).  For parity tests and bandwidth timing. */
mpcg_status mpcg_spmv(mpcg_ctx *ctx, const mpcg_csr *A, int32_t precision, const void *x, void *y);

/* Breadth-first search from vertex src over the stored pattern (self-loops
 * ignored).  dist: device int32[n], -1 for unreached vertices.  *ecc (host)
 * gets the largest distance, *far (host) the smallest vertex at that distance. */
mpcg_status mpcg_bfs(mpcg_ctx *ctx, const mpcg_csr *A, int64_t src, int32_t *dist, int64_t *ecc,
                     int64_t *far);

/* Algorithm I with the Jacobi method in place of CG (the section on the
 * matrix graph diameter and rounding-error growth in other iterative
 * methods): x_{k+1} = D^{-1}(b - (L + U) x_k) with A = L + D + U, first in
 * FP32 on the FP32 copy of A and b from x0 = 0 until the FP32 residual
 * ||b - A x_k|| <= eps1 ||b|| (or maxit1 updates: MPCG_FLAG_FP32_MAXIT, the
 * "cannot be achieved" entries of the paper's Jacobi table), then in FP64 from
 * float64(x~) until ||b - A x_k|| <= eps2 ||b||.  Each iteration forms
 * s = sum_{j != i} a_ij x_j (row order, one fma chain), t = b_i - s, the
 * residual t - a_ii x_i of the iterate and x_{k+1,i} = t / a_ii.
 *
 * A, b, x as for mpcg_solve; eps1 > 0 or MPCG_EPS1_NONE (FP64 only; kNN eps1
 * is not offered); eps2 > 0.  stats: n1, n2 = updates per stage, relres_sp =
 * the FP32 stage's last residual / ||b||, relres_final_true = the FP64
 * residual of the returned x / ||b||, flags, status.  A missing or
 * non-positive diagonal entry is ENOTSPD (Jacobi divides by a_ii).  Returns
 * OK, ENOCONV (maxit2 reached; x holds the last iterate), ENONFINITE or an
 * input error as mpcg_solve. */
mpcg_status mpcg_solve_jacobi(mpcg_ctx *ctx, const mpcg_csr *A, const double *b, double *x, double eps1,
                              double eps2, mpcg_stats *stats);

/* Multi-start 2BFS and an effective-diameter estimate.  The section on
 * computing the pseudo-diameter notes that repeating 2BFS from several start
 * vertices and keeping the largest pseudo-diameter improves the estimate;
 * Remark 1 relates it to the effective diameter, the distance within which a
 * fixed share q (typically 0.9) of the vertex pairs lie.
 *
 * starts: host int32[count], each 0 <= s < n (count may be 0).
 * q:      the share, 0 < q <= 1.
 * out (host):
 *   pdiam        the standard 2BFS pseudo-diameter (per component,
 *                maximised), as mpcg_features reports it;
 *   pdiam_multi  the largest of pdiam and, for each start s, l(t_s, u_s):
 *                t_s the vertex farthest from s, u_s the vertex farthest from
 *                t_s (ties: smallest index) -- a 2BFS inside s's component;
 *   best_start   index into starts of the first start whose 2BFS exceeded
 *                every value before it, -1 when pdiam_multi == pdiam;
 *   eff_diam     the smallest d >= 1 such that at least q of the pairs
 *                (s, v) -- s a start, v reachable from s, v != s -- have
 *                distance <= d (compared as cum >= q * pairs in double);
 *                0 when there is no pair;
 *   pairs        the number of such pairs.
 * Overwrites the workspace.  EINVAL for a null pointer, a start out of range,
 * count < 0 or q outside (0, 1]. */
typedef struct {
    int64_t pdiam;
    int64_t pdiam_multi;
    int64_t eff_diam;
    int64_t pairs;
    int32_t best_start;
    int32_t pad_;
} mpcg_diam_t;

mpcg_status mpcg_diameter_multi(mpcg_ctx *ctx, const mpcg_csr *A, const int32_t *starts, int32_t count,
                                double q, mpcg_diam_t *out);

/* Scheduling parameters of the products and the 2BFS (the autotuner's
 * knobs).  None changes a result: each picks how a product issues its loads
 * or how many blocks expand a 2BFS level, never what is summed in which
 * order (the block partitions that fix the reduction order are constants of
 * the library).  Sources, in order: mpcg_set_tuning's values for every
 * matrix; else the entry of the table loaded with mpcg_load_tuning for the
 * matrix's class (GPU architecture and compute units, 16- or 32-bit SELL
 * column offsets, round(log2(nnz / n)), nearest floor(log2(n))); else the
 * built-in defaults.  mpcg_options.spmv_variant 1-3 and bfs_mode 1-2 override
 * sell_split, the SELL/CSR choice and bfs_persist. */
typedef struct {
    int32_t sell_batch;          /* SELL-64 entries of a row whose loads are issued together: 4 or 8 */
    int32_t sell_whole_batch;    /* bit 0 FP32, bit 1 FP64 products: every lane loads its whole batch
                                    (slice padding included) instead of guarding each entry */
    int32_t sell_split;          /* CG product in two launches: 0 no, 1 yes, -1 for 32-bit columns */
    int32_t bfs_grid;            /* blocks of the 2BFS level kernel, 1..4096 */
    int32_t bfs_grid_shared;     /* the same beside Algorithm II's FP32 phase, 1..4096 */
    int32_t bfs_persist;         /* 1: large 2BFS levels in one persistent launch */
    int32_t batch_group_steps;   /* batch engine: steps enqueued per group, 1..64 */
    int32_t batch_bfs_rounds;    /* 2BFS rounds per pass of its BFS stream, 1..64 */
    int32_t batch_small_cap;     /* largest frontier one block per system expands, 1..2048 */
    int32_t batch_small_levels;  /* levels one such launch may expand, 1..4096 */
    int32_t batch_level_grid;    /* blocks of the multi-block level kernel, 1..65536 */
    int32_t bfs_dia;             /* 2BFS sweeps as bit-parallel levels over the diagonals when the
                                    pattern lies on at most 16 of them: 0 never, 1 when the pattern is
                                    wider than |i - j| <= 8 and has at least 2^16 rows, 2 whenever it
                                    qualifies */
    int32_t bfs_dia_tiles;       /* with bfs_dia: 1 = several levels per launch (a block forms them on
                                    its own words plus a halo that the levels consume: up to 16 levels
                                    per tile where 8 or more fit, else 2 per launch), 0 = one launch
                                    per level */
    int32_t sell_stream;         /* the SELL products read the matrix with nontemporal loads: -1 where
                                    that precision's copy exceeds the 256 MB Infinity Cache, 0 never,
                                    1 always */
    int32_t batch_runahead;      /* batch engine, Algorithm II, a system whose features are still
                                    being computed: 1 = it runs ahead in FP32 with copies of x~ at
                                    each candidate's crossing and a speculative FP64 phase; 2 = it
                                    waits at its first crossing of a candidate, taking no bandwidth
                                    from the others; 0 = it waits while more than 8 systems share
                                    the steps, else runs ahead */
    int32_t batch_bfs_band;      /* batch engine: 1 = a connected system whose pattern lies within
                                    |i - j| <= 31 takes its 2BFS as bit-parallel levels of one wave
                                    per system, 0 = the level kernels of every other system */
} mpcg_tuning;

/* Use *t for every matrix from now on (NULL: back to the table and the
 * defaults).  EINVAL for a value out of range.  The batch engine takes its
 * fields when mpcg_batch_set_workspace starts it. */
mpcg_status mpcg_set_tuning(mpcg_ctx *ctx, const mpcg_tuning *t);

/* Load a tuning table (host path; text, header "mpcg-tune 1", then lines
 * "solve <arch> <cu> <idx16> <lenlog> <nlog> <sell_batch> <sell_whole_batch>
 * <sell_split> <bfs_grid> <bfs_grid_shared> <bfs_persist> [<bfs_dia> [<bfs_dia_tiles> [<sell_stream>]]]" and at most one
 * "batch <arch> <cu> <group_steps> <bfs_rounds> <small_cap> <small_levels>
 * <level_grid> [<runahead> [<bfs_band>]]").  EINVAL for a missing or
 * malformed file (the previous table is kept). */
mpcg_status mpcg_load_tuning(mpcg_ctx *ctx, const char *path);

/* The parameters a solve would use for a matrix of n rows, nnz entries and
 * largest |i - j| = band (HOST output). */
mpcg_status mpcg_get_tuning(const mpcg_ctx *ctx, int64_t n, int64_t nnz, int64_t band, mpcg_tuning *out);

/* Time of the most recent mpcg_spmv kernel launch in milliseconds (HIP events
 * on the context stream), 0 if none. */
mpcg_status mpcg_last_kernel_ms(const mpcg_ctx *ctx, double *ms);

/* Kernels that mpcg_time_kernel can time (the ones a solve launches). */
#define MPCG_KERNEL_CG_SPMV_F64 0   /* previous x += alpha d, direction update, q = A d, d.q; FP64
                                       (two launches, direction then product, for a matrix whose
                                       column offsets exceed 16 bits; timed together) */
#define MPCG_KERNEL_CG_SPMV_F32 1   /* the same on float32(A), FP32 vectors */
#define MPCG_KERNEL_UPDATE_F64 2    /* alpha, r -= alpha q, r.r; FP64 */
#define MPCG_KERNEL_UPDATE_F32 3
#define MPCG_KERNEL_SPMV_F64 4      /* plain y = A x (mpcg_spmv) */
#define MPCG_KERNEL_SPMV_F32 5
#define MPCG_KERNEL_JACOBI_F64 6    /* one Jacobi iteration of mpcg_solve_jacobi (residual + update), FP64 */
#define MPCG_KERNEL_JACOBI_F32 7

/* Measurement hook: run `reps` back-to-back launches of one solver kernel on A
 * with the workspace's scratch vectors (set to finite values, recurrence held
 * live), bracketed by HIP events on the context stream; *ms gets the mean
 * milliseconds per launch.  Overwrites the workspace only.  EINVAL for an
 * unknown kernel id or reps < 1. */
mpcg_status mpcg_time_kernel(mpcg_ctx *ctx, const mpcg_csr *A, int32_t kernel, int32_t reps,
                             double *ms);

const char *mpcg_strerror(mpcg_status s);

/* ------------------------------------------------------------------------
 * Batched and continuously admitted solves.
 *
 * Many independent systems are solved together: each admitted system gets a
 * range of 64-row slices and SELL-64 entries in the batch arena, and every
 * "step" advances all of them at once (CG product, scalar decisions, update,
 * 2BFS levels) with per-system reductions and per-system convergence, so a
 * system's result does not depend on the other systems it shares the GPU
 * with.  Each system follows Algorithm I (fixed eps1), Algorithm II
 * (MPCG_EPS1_AUTO: 2BFS per connected component and the k0 prefix run side by
 * side, then kNN) or FP64-only CG (MPCG_EPS1_NONE), with the restart and final
 * check of mpcg_solve.  Requests that arrive while others run are admitted as
 * slots, slices and entries free up (first fit), and their work joins the
 * next step.  A host thread owned by the context drives the steps on a
 * stream of its own; mpcg_batch_poll returns finished solves without blocking.
 *
 * Its scheduling knobs (steps per group, 2BFS rounds, the one-block 2BFS
 * kernel's frontier and level caps, the level kernel's grid) are the batch_*
 * fields of mpcg_tuning, taken when the engine starts; none changes any
 * result, only when work runs.
 * -------------------------------------------------------------------------*/

/* One solve.  A, b and x are DEVICE memory owned by the caller and borrowed
 * until mpcg_batch_poll has reported the request: A and b must stay
 * unchanged and complete (the caller's stream synchronised) at submission; x
 * (n doubles) receives the solution. */
typedef struct {
    mpcg_csr A;
    const double *b;
    double *x;
    double eps1;       /* MPCG_EPS1_AUTO, MPCG_EPS1_NONE or a finite value > 0 */
    double eps2;       /* > 0 */
    void *user;        /* not used by the library */
} mpcg_request;

/* Arena bytes for a batch engine holding at most max_systems systems,
 * max_rows rows in total (each system is padded to a multiple of 64 rows) and
 * max_entries SELL-64 entries in total (nnz plus padding to the longest row
 * of each 64-row slice).  EINVAL for non-positive sizes. */
mpcg_status mpcg_batch_workspace_size(const mpcg_ctx *ctx, int64_t max_rows, int64_t max_entries,
                                      int32_t max_systems, size_t *bytes);
/* Hands a device arena (>= the size above, 256-byte aligned, owned by the
 * caller until mpcg_destroy) to the batch engine of this context and starts
 * its host thread.  Once per context; EBUSY if the engine already runs. */
mpcg_status mpcg_batch_set_workspace(mpcg_ctx *ctx, void *dev_arena, size_t bytes, int64_t max_rows,
                                     int64_t max_entries, int32_t max_systems);
/* Queues `count` requests; ids[i] (HOST array) receives the id of reqs[i].
 * Validated before anything is queued: EINVAL (bad sizes, pointers or
 * tolerances), ENOMODEL (AUTO without a model), ENOMEM (a system larger than
 * the whole arena), EDEVICE (no engine).  Malformed CSR contents are
 * reported per request by mpcg_batch_poll (EINVAL / ENONFINITE). */
mpcg_status mpcg_batch_submit(mpcg_ctx *ctx, const mpcg_request *reqs, int32_t count, uint64_t *ids);
/* Non-blocking: moves up to `cap` finished requests out of the engine;
 * done_ids[i] and done_stats[i] (HOST arrays) describe one of them, with its
 * own status in done_stats[i].status; *n_done gets the count.  Before a
 * request is reported its x is complete in device memory. */
mpcg_status mpcg_batch_poll(mpcg_ctx *ctx, uint64_t *done_ids, mpcg_stats *done_stats, int32_t cap,
                            int32_t *n_done);
/* Cancels a queued or running request; it is reported by mpcg_batch_poll
 * with status ECANCELED (x undefined).  EINVAL for an unknown or finished id. */
mpcg_status mpcg_batch_cancel(mpcg_ctx *ctx, uint64_t id);
/* Requests waiting for admission and systems on the GPU (HOST outputs). */
mpcg_status mpcg_batch_load(mpcg_ctx *ctx, int32_t *queued, int32_t *active);

#ifdef __cplusplus
}
#endif

#endif /* MPCG_H */
