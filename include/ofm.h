/*
 * ofm.h -- C ABI of the MI355X (gfx950) orthogonalization-free spectral
 * clustering library (libofm.so).
 *
 * The library computes low-dimensional spectral features of an undirected
 * graph without any orthogonalization, by running the gradient-type iteration
 * of Pang & Yang, "Spectral clustering via orthogonalization-free methods"
 * (arXiv 2305.10356), on the shifted normalized Laplacian A = L - 2I, and
 * provides the post-processing of its Algorithm 1 (row normalisation and the
 * K-means assignment step).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers are DEVICE pointers unless a parameter name starts with "host_".
 * - The caller owns every array it passes in; the library never frees them.
 *   Handles (ofm_laplacian, ofm_workspace) own only library-allocated memory.
 * - Dense feature blocks (X, Z, Y, V, G) are N x k, row-major (C-contiguous),
 *   FP64 for OFM_FP64 and FP32 for OFM_FP32.  Supported widths:
 *   k in {4, 8, 16, 32, 64}.  (Zero columns are fixed points of every
 *   variant and never influence the other columns, and the residual leaves
 *   exactly zero columns out, so a block of another width can be zero-padded
 *   to the next supported one.)
 * - Graph indices are int32 (nnz < 2^31).
 * - All work is enqueued on the given HIP stream (0 = null stream) and is
 *   asynchronous unless the comment says "synchronizing".  No entry point
 *   synchronizes the device as a whole.  Handles are not thread-safe.
 * - Every entry point returns an ofm_status and never throws.  Argument and
 *   shape errors are detected on the host before anything is enqueued.
 *   Numerical failures detected on the device (non-finite values, Cholesky
 *   failure in the residual, a line search without a real root) set a device
 *   status word that the next synchronizing call (ofm_solve, ofm_get_stats)
 *   returns; when several are set: OFM_E_NONFINITE, then OFM_E_NUMERIC, then
 *   OFM_E_NO_ROOT.
 */
#ifndef OFM_H
#define OFM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ofm_status {
  OFM_OK = 0,
  OFM_E_INVALID_ARG = -1,  /* null pointer, negative size, bad enum value   */
  OFM_E_SHAPE = -2,        /* unsupported k, k > N, mismatched sizes        */
  OFM_E_GRAPH = -3,        /* malformed CSR, column out of range, a node of
                              zero degree, or (with OFM_LAP_VALIDATE) a
                              pattern that is not symmetric                  */
  OFM_E_NONFINITE = -4,    /* NaN/Inf met in a Gram, a step size or beta     */
  OFM_E_NUMERIC = -5,      /* X^T X not positive definite in the residual   */
  OFM_E_HIP = -6,          /* a HIP runtime call failed                      */
  OFM_E_NOMEM = -7,        /* device allocation failed                       */
  OFM_E_UNSUPPORTED = -8,  /* option combination not implemented             */
  OFM_E_NO_ROOT = -9       /* a line-search cubic that is not identically
                              zero had no real root (Section 3.2 gives no rule
                              for it): that step took step size 0            */
} ofm_status;

/* The four methods (Introduction and Section 2):
 *   OFM_F1     gradient of f1(X) = ||A + X X^T||_F^2      (eq. gradientf1)
 *   OFM_TRI_F1 g1(X) = A X + X triu(X^T X)                 (eq. gradientg1)
 *   OFM_F2     gradient of f2(X) = tr((2I - X^T X) X^T A X) (eq. gradientf2)
 *   OFM_TRI_F2 g2(X) = 2AX - AX triu(X^T X) - X triu(X^T A X) (eq. gradientg2) */
typedef enum ofm_variant { OFM_F1 = 0, OFM_TRI_F1 = 1, OFM_F2 = 2, OFM_TRI_F2 = 3 } ofm_variant;

/* Arithmetic of the N x k passes.  k x k products (Grams), step sizes, beta
 * and the residual are FP64 in both modes.
 *   OFM_FP64: X, SpMM accumulation and the N x k updates in FP64.
 *   OFM_FP32: X in FP32; SpMM with FP32 edge weights and FP32 accumulation;
 *             N x k updates in FP32; Grams accumulated in FP64 from the FP32
 *             values (every product exact). */
typedef enum ofm_precision { OFM_FP64 = 0, OFM_FP32 = 1, OFM_FP32_BF16X = 2 } ofm_precision;
/*   OFM_FP32_BF16X (workspaces only): as OFM_FP32, but the SpMMs of the
 *             iteration gather the neighbour rows from a BF16 copy of X (and of
 *             V) kept by the workspace (round to nearest even); the row's own
 *             term and every other pass stay FP32.  Halves the bytes of the
 *             random row gathers; the reachable residual is limited to about
 *             the BF16 rounding (~1e-3).  ofm_residual and ofm_objective use
 *             the FP32 rows. */

/* ofm_build_laplacian flags */
#define OFM_LAP_VALIDATE 1u   /* also check that the pattern is symmetric    */
#define OFM_LAP_NO_REORDER 2u /* process rows in index order, not by degree  */
#define OFM_LAP_NO_UPPER 4u   /* build no upper-triangle copy (see below)     */

typedef struct ofm_laplacian_s* ofm_laplacian;
typedef struct ofm_workspace_s* ofm_workspace;

typedef struct ofm_opts {
  int variant;      /* ofm_variant                                            */
  int precision;    /* ofm_precision                                          */
  int max_iter;     /* ofm_solve: maximum number of X updates (>= 1)          */
  int check_every;  /* residual computed every check_every updates (>= 1)     */
  int first_step;   /* 0: exact line search for the update before the loop of
                       Algorithm 2; 1: use alpha0 (the algorithm's input step) */
  int restart;      /* 1: descent restart, beta_i := 0 when <V_i, G_i> >= 0
                       (a safeguard outside Algorithm 2; 0 = as printed)      */
  double alpha0;    /* step for first_step = 1                                */
  double tol;       /* ofm_solve stops when the residual <= tol (0: never)    */
  int graph;        /* ofm_solve: 1 = run the loop as replays of a HIP graph
                       holding check_every updates (captured on first use on
                       a stream of the workspace; see ofm_solve); 0 = eager   */
  int recur;        /* 0: two products with A per update, A X^t and A V^t, as
                       Algorithm 2 is costed (Table 1).  1: A X^{t+1} =
                       A X^t + A V^t diag(alpha^t) by recurrence, with A X
                       recomputed exactly at every residual evaluation (every
                       check_every updates), after ofm_init / ofm_set_state
                       and after ofm_residual / ofm_objective; one product
                       with A per update in between.  Same iteration in exact
                       arithmetic; rounding differs.  Needs one more N x k
                       buffer (A V).                                          */
  int gather;       /* cache policy of the row gathers of the products with A:
                       1: default; 2: hot/cold, rows of the less connected
                       columns (below the top fifth of rows by entry count,
                       marked when the Laplacian is built) loaded
                       non-temporally so that they do not evict the rows
                       gathered most often; 0: time both once at
                       ofm_workspace_create and keep the faster (only when
                       the N x k block is at least 32 MB, else 1).  Results
                       are bitwise the same.  2 is refused (OFM_E_UNSUPPORTED)
                       for OFM_FP32_BF16X and for blocks of 2 GB or more.
                       The batched solver always uses 1.                      */
  double freeze_eps; /* > 0: a step whose direction is negligible against the
                       iterate, ||G||_F <= freeze_eps ||X||_F (G = g(X^t) of
                       the step, X^t the iterate entering it), takes step size
                       0 in every column, so a converged X stays where it is
                       instead of drifting with the rounding noise (Algorithm 2
                       itself runs a fixed number of steps).  0 = off.        */
} ofm_opts;

typedef struct ofm_stats {
  int64_t iters;     /* number of X updates done since ofm_init               */
  int32_t status;    /* ofm_status of the device status word                  */
  int32_t converged; /* 1 when the last residual <= tol                       */
  double relres;     /* last residual ||A U - U Lam||_F / ||U Lam||_F of the Ritz
                        pairs (Lam, U) of A on span(X), numerical results
                        section "Evaluation metrics"; computed from X^T X,
                        X^T A X and (AX)^T (AX) without orthogonalization;
                        -1 if none was computed yet                           */
  double objective;  /* f1 or f2 at the X of the last residual                */
  int64_t relres_iter; /* iteration whose X the residual belongs to           */
  int32_t gather;    /* gather policy in use (1 default, 2 hot/cold)          */
  int32_t reserved;
} ofm_stats;

/* Human-readable name of a status code (static string). */
const char* ofm_status_string(int status);

/* Library version string (static). */
const char* ofm_version(void);

/*
 * Build the shifted normalized Laplacian A = L - 2I = -I - D^{-1/2} S D^{-1/2}
 * (Introduction, eq. (1); Algorithm 1, step 2) of an undirected graph given as
 * a CSR similarity matrix S (both directions of every edge stored).
 *   n, nnz      number of nodes and of stored entries
 *   row_ptr     int32[n+1], row_ptr[0] = 0, row_ptr[n] = nnz, non-decreasing
 *   col_idx     int32[nnz], entries in [0, n)
 *   vals        nullable: NULL means S_ij = 1 for every stored entry;
 *               otherwise nnz weights S_ij >= 0 (must be symmetric) of type
 *               vals_dtype; self-loops (i == j) count once in D_ii
 *   vals_dtype  OFM_FP64 (double) or OFM_FP32 (float, widened exactly to
 *               FP64 before any arithmetic); ignored when vals is NULL
 *   flags       OFM_LAP_VALIDATE, OFM_LAP_NO_REORDER, OFM_LAP_NO_UPPER
 * Computes D_ii = sum_j S_ij, D^{-1/2}, ||A||_F^2 and the normalized edge
 * weights w_ij = D_ii^{-1/2} S_ij D_jj^{-1/2} (FP64 and FP32 copies, laid out
 * in the row-processing order).  Synchronizing (the checks are read back).
 * Upper-triangle copy: unless OFM_LAP_NO_UPPER or OFM_LAP_NO_REORDER is given
 * or some row has a self-loop, an upper-triangle copy is also packed: of every
 * stored pair (i, j), (j, i) the entry whose column j comes later in the order
 * of the nodes by (degree, id) (half of nnz, 24 B per entry for the FP32 and
 * FP64 copies together), rows by their count of such entries, descending (in
 * the grouped order for ofm_build_laplacian_grouped).  With A symmetric and
 * U_i = sum over row i of the copy of w_ij V_j, the line searches' products
 * with A V (Section 3.2) are diag(V^T A V) = -diag(V^T V) - 2 diag(V^T U),
 * V^T A V = -V^T V - V^T U - U^T V and X^T A V = (AX)^T V: a workspace on such
 * a Laplacian gathers only the copy's entries for them (half the gathers of
 * the product A V, and those go to the rows of larger degree).  The symmetry of the pattern and the weights
 * that the method assumes is then also what the step relies on
 * (OFM_LAP_VALIDATE checks it).
 * The input arrays are only read during the call.
 * Errors: OFM_E_GRAPH for a malformed CSR, an out-of-range column, a zero
 * degree or (when validating) an asymmetric pattern.
 */
ofm_status ofm_build_laplacian(int64_t n, int64_t nnz, const int32_t* row_ptr,
                               const int32_t* col_idx, const void* vals, int vals_dtype,
                               unsigned flags, hipStream_t stream, ofm_laplacian* out);

/*
 * As ofm_build_laplacian, with a row-processing order laid out for the eight
 * XCDs of the chip (each with its own L2) from a grouping of the nodes, such as
 * the cluster labels of an earlier solve of the same or a previous snapshot of
 * the graph (Algorithm 1, step 5; the streaming experiments of the numerical
 * results section start each stage from the previous one).  The groups are
 * dealt to eight slots, balancing their entry counts; every SpMM then runs the
 * rows of slot x on the workgroups that the hardware places on XCD x (workgroup
 * ids congruent to x modulo 8), a group at a time, so that the neighbour rows a
 * community gathers stay in that XCD's L2.  Within a slot: the rows processed a
 * wavefront per row (64 or more entries) first, then group by group, each by
 * entry count, descending.
 *   host_groups  host int32[n]: group of each node; any negative value means
 *                "no group" (such rows are dealt to the slots last).  Values
 *                must be < n.  Only read during the call.
 * Results of ofm_apply_A are bitwise those of ofm_build_laplacian's order; the
 * k x k products of a workspace are summed over other workgroup partitions
 * (differences at the rounding of the FP64 sums).  Products with A on such a
 * Laplacian launch one workgroup per few 16-row tiles of each slot (tens of
 * thousands of workgroups for millions of rows); a workspace created on it
 * therefore holds more reduction scratch: 3k doubles per workgroup of its
 * largest such grid (about 3k doubles per 32 to 64 rows, e.g. 24 MB at
 * N = 2M, k = 32, FP32).
 * Errors: as ofm_build_laplacian; OFM_E_INVALID_ARG for a null host_groups, a
 * group id >= n, or OFM_LAP_NO_REORDER in flags.
 */
ofm_status ofm_build_laplacian_grouped(int64_t n, int64_t nnz, const int32_t* row_ptr,
                                       const int32_t* col_idx, const void* vals, int vals_dtype,
                                       unsigned flags, const int32_t* host_groups,
                                       hipStream_t stream, ofm_laplacian* out);

/*
 * The row-processing order that ofm_build_laplacian_grouped lays out, computed
 * on the host alone (no device call): host_order (int32[n]) receives the rows
 * in processing order, host_slot_start (int64[9]) the first position of each
 * of the eight XCD slots and n.  host_row_ptr is the CSR row_ptr (int32[n+1]),
 * host_groups as for ofm_build_laplacian_grouped.  For inspecting or reusing
 * the order (e.g. to lay out other per-node data the same way).
 * Errors: OFM_E_INVALID_ARG for null pointers, n <= 0 or a group id >= n;
 * OFM_E_GRAPH for a row_ptr that does not start at 0 or decreases.
 */
ofm_status ofm_grouped_order(int64_t n, const int32_t* host_row_ptr, const int32_t* host_groups,
                             int32_t* host_order, int64_t* host_slot_start);

ofm_status ofm_laplacian_destroy(ofm_laplacian lap);

/* Host copies of the basic graph quantities: n, nnz, ||A||_F^2, and (nullable
 * outputs) the degrees D_ii as FP64[n] into host_degrees. Synchronizing. */
ofm_status ofm_laplacian_info(ofm_laplacian lap, int64_t* host_n, int64_t* host_nnz,
                              double* host_normA2, double* host_degrees);

/* Size of the upper-triangle copy (see ofm_build_laplacian): its rows (those
 * with at least one entry in it) and entries; both 0 when none was built.  Either output may be NULL.  Errors: OFM_E_INVALID_ARG for a null
 * handle. */
ofm_status ofm_laplacian_upper(ofm_laplacian lap, int64_t* host_rows, int64_t* host_nnz);

/*
 * Y = A Z for an N x k block Z (the sparse-times-tall-skinny product of the
 * iteration, Section 3.3 eq. spmm with the shift of Algorithm 1).
 * Z and Y must not overlap.  precision selects FP64 or FP32 storage and
 * arithmetic as described at ofm_precision.
 */
ofm_status ofm_apply_A(ofm_laplacian lap, int k, int precision, const void* Z, void* Y,
                       hipStream_t stream);

/*
 * Create the iteration workspace: the direction and CG buffers V, V_prev, G,
 * G_prev, AX, AV (with the recurrence, and for the f2 variants at k >= 32),
 * the k x k FP64 products and the reduction scratch.  Allocates device memory
 * (5 or 6 N x k blocks, plus BF16 copies of X and V for OFM_FP32_BF16X, plus
 * O(k^2) per workgroup of the passes; on a Laplacian from
 * ofm_build_laplacian_grouped, 3k doubles per 32 to 64 rows).  host_opts is
 * copied.  With opts.gather = 0 and a block
 * of 32 MB or more it also runs and times six products with A (synchronizing).
 */
ofm_status ofm_workspace_create(ofm_laplacian lap, int k, const ofm_opts* host_opts,
                                ofm_workspace* out);
ofm_status ofm_workspace_destroy(ofm_workspace ws);

/*
 * Algorithm 2 before its loop: G0 = g(X0), V0 = -G0, step size (exact line
 * search, or alpha0 when first_step = 1), X1 = X0 + V0 diag(alpha).
 * X (N x k, in/out) is updated in place.  Resets the iteration counter to 1.
 */
ofm_status ofm_init(ofm_workspace ws, void* X, hipStream_t stream);

/*
 * One loop iteration of Algorithm 2 on X (in/out, N x k):
 *   G = g(X);  beta_i = sum_r (G - G_prev)_ri G_ri / sum_r G_prev,ri^2
 *   (beta_i = 0 when the denominator is 0);  V_i = -G_i + beta_i V_prev,i;
 *   exact line search (Section 3.2): the cubic of eq. f1-derivative /
 *   f2-derivative (one step for all columns) or of eq. alphai-f1 /
 *   alphai-f2 (one step per column), real roots by Cardano's formula and
 *   the root rules of Section 3.2 (the triangular variants take the real root
 *   of smallest |alpha| when there are three);  X_i += alpha_i V_i.
 * Every check_every iterations it also computes the residual of X^t (the
 * iterate entering the step).  Enqueues kernels only: no host
 * synchronization and no allocation, so the call can be captured in a HIP
 * graph (once ofm_init has run).
 */
ofm_status ofm_step(ofm_workspace ws, void* X, hipStream_t stream);

/*
 * ofm_init, then ofm_step until the residual <= tol or max_iter updates.
 * Synchronizing: reads the stats every check_every iterations.  When tol > 0,
 * a residual evaluation that meets tol freezes X on the device (every later
 * step size is 0 until the next ofm_init / ofm_set_state), so the returned X
 * is the iterate whose residual was reported.
 * With opts.graph = 1 the updates between two residual evaluations (the
 * check_every ofm_step calls that end with one) are captured once into a HIP
 * graph and replayed; the kernels and their arguments are those of the eager
 * loop, so the result is bitwise the same.  The graph is captured for the X
 * pointer of the call (and the buffer parity of the step state) and kept by
 * the workspace; a call with another X captures again.  Per-pass timing
 * (ofm_set_timing) does not see replayed passes.
 */
ofm_status ofm_solve(ofm_workspace ws, void* X, hipStream_t stream, ofm_stats* host_out);

/* Residual and objective of X now (enqueues the products, then reads back).
 * Synchronizing. */
ofm_status ofm_residual(ofm_workspace ws, const void* X, hipStream_t stream, ofm_stats* host_out);

/* Copy of the current stats and device status word. Synchronizing. */
ofm_status ofm_get_stats(ofm_workspace ws, hipStream_t stream, ofm_stats* host_out);

/*
 * CG state exchange (checkpoint / resume, and step-by-step comparison).
 * ofm_get_state copies V^{t-1} and G^{t-1} (N x k each, workspace precision)
 * into caller buffers.  ofm_set_state loads them from caller buffers, sets the
 * iteration counter to t (>= 1) and recomputes the products of X the next
 * step needs; the next ofm_step then continues from (X, V_prev, G_prev).
 */
ofm_status ofm_get_state(ofm_workspace ws, void* V_prev, void* G_prev, hipStream_t stream);
ofm_status ofm_set_state(ofm_workspace ws, const void* X, const void* V_prev,
                         const void* G_prev, int64_t t, hipStream_t stream);

/*
 * Scalars of the last step (synchronizing); any host pointer may be NULL.
 *   host_alpha  double[k] step sizes (all equal for OFM_F1 / OFM_F2)
 *   host_beta   double[k] CG coefficients (0 for the step before the loop)
 *   host_coef   double[4*k] cubic coefficients (a3, a2, a1, a0) per column:
 *               host_coef[4*i + j]; the OFM variants store their single cubic
 *               in column 0
 *   host_nroots int32[k] number of real roots found
 */
ofm_status ofm_get_step_info(ofm_workspace ws, double* host_alpha, double* host_beta,
                             double* host_coef, int32_t* host_nroots, hipStream_t stream);

/*
 * The root rules of the exact line search (Section 3.2; the device code every
 * step runs) applied to caller-given cubics, for checking them in isolation:
 * coef FP64[4*count], coef[4*i + j] = a_{3-j} of cubic i, a3 x^3 + a2 x^2 +
 * a1 x + a0 (device).  alpha FP64[count] receives the chosen real root (0 when
 * there is none), nroots int32[count] the number of distinct real roots found
 * (0 to 3).  variant selects the rule among three real roots: the least line
 * objective a3 x^4/4 + a2 x^3/3 + a1 x^2/2 + a0 x (OFM_F1, OFM_F2) or the
 * smallest |x| (OFM_TRI_F1, OFM_TRI_F2).  Asynchronous.
 * Errors: OFM_E_INVALID_ARG for a bad variant, count < 0 or a null pointer.
 */
ofm_status ofm_select_roots(int variant, int64_t count, const double* coef, double* alpha,
                            int32_t* nroots, hipStream_t stream);

/*
 * Memory-system measurement, not part of the method: Y_r = sum_e Z[idx[r S + e]]
 * for r < nrows, e < S, with rows of row_floats FP32 values (16, 32 or 64:
 * 64, 128 or 256 bytes; Z: zrows rows, Y: nrows rows, row-major).  This is the
 * row-gather pattern of the products with A without their sparse-matrix
 * bookkeeping, for measuring how fast the chip serves random rows (bench.py
 * --gather-ceiling).  idx: int32[nrows * S], every value in [0, zrows) (not
 * checked).  Asynchronous.
 * Errors: OFM_E_INVALID_ARG for null pointers or sizes below 1; OFM_E_SHAPE for
 * another row width.
 */
ofm_status ofm_gather_rows(int64_t nrows, int S, int row_floats, const int32_t* idx,
                           const float* Z, int64_t zrows, float* Y, hipStream_t stream);

/*
 * Batched solves of many independent graphs (any sizes, widths k in
 * {4, 8, 16, 32, 64}): Algorithm 2 runs on all of them in lockstep, each pass
 * being one launch per width group over every graph of the group; a graph
 * stops iterating (on the device) as soon as its residual meets tol.
 * host_laps[count], host_ks[count]: the graphs and their widths (the handles
 * must outlive the batch); host_opts: shared options (precision OFM_FP32 or
 * OFM_FP32_BF16X; variant, max_iter, check_every, tol, restart, first_step,
 * recur, freeze_eps; graph = 1 runs the lockstep loop of ofm_batch_solve, after
 * the schedule has been chosen, as replays of one HIP graph per check_every
 * updates of every graph; the FP64 finishing solves always run eagerly).
 * Allocates the per-graph state (with tol > 0 also a copy of the starting
 * block of every graph with k <= 32, for the finishing solves below).  The block schedule (each graph's blocks on
 * one XCD; a target of tiles per wavefront, 2, 4, 8 or 16, which sets the
 * blocks per graph, and at most 128 or 64 blocks per XCD) is chosen among these
 * eight candidates by timing the first iterations of the first solve (the GPU
 * time from the first width group's start to the last one's end, HIP events)
 * and kept for later solves (see ofm_batch_set_schedule).
 */
typedef struct ofm_batch_s* ofm_batch;
ofm_status ofm_batch_create(int count, const ofm_laplacian* host_laps, const int* host_ks,
                            const ofm_opts* host_opts, ofm_batch* out);
ofm_status ofm_batch_destroy(ofm_batch b);
/* Solve every graph from its X (host_X[i]: device pointer to graph i's N_i x k_i
 * FP32 block, updated in place); host_stats[count] receives the per-graph
 * stats (iters = updates done, relres of the X it stopped at).  A graph whose
 * FP32 residual decreases by less than 5% over 10 checks before reaching tol
 * (or that reaches max_iter) is finished in FP64 (k <= 32) by two solves that
 * race, one from its FP32 X with a fresh CG state and one from its starting
 * block: the first to reach tol wins (the other stops at its next residual
 * check), and with none the first one's result is kept.  That stage allocates
 * a workspace per solve and runs up to 4 of them at once, each on its own
 * stream and host thread, once the FP32 loop has ended.  Synchronizing. */
ofm_status ofm_batch_solve(ofm_batch b, void* const* host_X, hipStream_t stream,
                           ofm_stats* host_stats);
/*
 * The lockstep iteration one step at a time (checkpoint / resume, and
 * step-by-step comparison): ofm_batch_init runs the set-up step of Algorithm 2
 * on every graph (host_X as for ofm_batch_solve; the blocks must stay the same
 * until the next ofm_batch_init) and marks every graph active; ofm_batch_step
 * runs one loop iteration of Algorithm 2 on every active graph, with the
 * residual every check_every updates (a graph whose residual meets tol stops
 * iterating, as in the solve; no FP64 finishing), on the schedule chosen by the
 * last solve (the first candidate before any).  ofm_batch_init synchronizes the
 * batch's streams; ofm_batch_step only enqueues.
 */
ofm_status ofm_batch_init(ofm_batch b, void* const* host_X, hipStream_t stream);
ofm_status ofm_batch_step(ofm_batch b, hipStream_t stream);
/* Graph i's CG state V^{t-1}, G^{t-1} (N_i x k_i FP32 each) copied into
 * caller buffers, after ofm_batch_init / ofm_batch_solve. */
ofm_status ofm_batch_get_state(ofm_batch b, int i, void* V_prev, void* G_prev,
                               hipStream_t stream);
/* Scalars of graph i's last lockstep step, as ofm_get_step_info (synchronizing;
 * any host pointer may be NULL). */
ofm_status ofm_batch_get_step_info(ofm_batch b, int i, double* host_alpha, double* host_beta,
                                   double* host_coef, int32_t* host_nroots, hipStream_t stream);
/* Schedule of width group `group` (groups in increasing k; host_ngroups
 * receives their number): host_k its width, host_tpw the tiles per wavefront
 * target (blocks per graph ~ tiles / (waves per block * tpw)), host_workers
 * the blocks per XCD cap, host_ms[8] the measured GPU time of a whole batch
 * iteration with each candidate (tpw 2, 4, 8, 16 with 128 blocks per XCD, then
 * with 64; 0 if untried; every group runs the same candidate); host_escalated = number of graphs the last solve finished in FP64.
 * Any pointer may be NULL; an out-of-range group fills only host_ngroups and
 * host_escalated and returns OFM_E_INVALID_ARG. */
ofm_status ofm_batch_schedule(ofm_batch b, int group, int* host_ngroups, int* host_k,
                              int* host_tpw, int* host_workers, double* host_ms,
                              int* host_escalated);
/* Fix the block schedule of every width group to tpw tiles per wavefront
 * (2, 4, 8 or 16) with at most `workers` blocks per XCD (128 or 64, or any
 * count from 8 to 63, e.g. to match what a persistent launch keeps resident)
 * for the following solves and steps; tpw = 0 times the candidates again at
 * the next solve.  Errors: OFM_E_INVALID_ARG for another value. */
ofm_status ofm_batch_set_schedule(ofm_batch b, int tpw, int workers);
/* Host wall time of the last solve's two stages: the lockstep FP32 loop
 * (host_loop_ms, to the end of its last iteration) and what follows it
 * (host_finish_ms: the per-graph statistics and the FP64 finishing solves,
 * which run concurrently on up to 4 streams of the batch); host_replays: graph replays
 * of the lockstep loop (0 without opts.graph).  Any pointer may be NULL. */
ofm_status ofm_batch_phases(ofm_batch b, double* host_loop_ms, double* host_finish_ms,
                            int64_t* host_replays);
/* Persistent form of the lockstep loop: the batched iteration of Algorithm 2
 * as one launch per width group and chunk instead of one per pass.  on = 1: every check_every updates of the loop after the schedule timing run
 * as one cooperative launch per width group that walks the passes of an
 * update (SpMM of X with the direction, [residual], V pass, SpMM of V over the
 * upper-triangle copy, line search, update) with a grid-wide barrier after
 * each pass and after each of its per-graph reductions; the groups run one
 * after another on the solve's stream, each with as many workers per XCD as
 * its schedule gives and stay resident.  With the same workers per XCD the
 * iterates are bitwise those of the per-pass launches.  on = 0: per-pass
 * launches (eager or graph-replayed by opts.graph).  Supported for OFM-f1 and
 * TriOFM-f1, OFM_FP32, recur = 0, every k <= 32 (else OFM_E_UNSUPPORTED;
 * OFM_E_INVALID_ARG for on not 0 or 1).  A barrier wait beyond its spin limit
 * (2^24 polls) lets the launch run to its end and makes ofm_batch_solve return
 * OFM_E_HIP.  Allocates two small device words on the first call with on = 1. */
ofm_status ofm_batch_set_persistent(ofm_batch b, int on);
/* Persistent launches of the last ofm_batch_solve and the fewest workers per
 * XCD any of them used (0 when none ran).  Either pointer may be NULL. */
ofm_status ofm_batch_persist_info(ofm_batch b, int64_t* host_launches, int* host_workers);

/*
 * Host copy (synchronizing) of one k x k FP64 product held by the workspace,
 * row-major into host_kxk[k*k]:
 *   0: X^T X   1: X^T A X   2: (AX)^T (AX)   3: V^T V   4: X^T V
 *   5: X^T A V 6: V^T A V
 * The values are those of the last pass that produced them (X^T X after an
 * update is that of the new X; (AX)^T (AX) is that of the last residual
 * evaluation; X^T A X for the f1 variants is that of the last residual
 * evaluation, for the f2 variants that of the current iterate: each update
 * advances it as H + E D + D E^T + D F D with E = X^T A V, F = V^T A V and
 * D = diag(alpha), and every residual evaluation recomputes it exactly).
 */
ofm_status ofm_get_products(ofm_workspace ws, int which, double* host_kxk, hipStream_t stream);

/*
 * Objective and gradient (Sections 2.1 and 2.2) for the differentiable
 * variants of the workspace:
 *   OFM_F1: f1(X) = ||A + X X^T||_F^2,            grad = 4AX + 4X X^T X
 *   OFM_F2: f2(X) = tr((2I - X^T X) X^T A X),    grad = 4AX - 2X X^T A X - 2AX X^T X
 * (eqs. gradientf1, gradientf2).  The triangular directions g1, g2 are not
 * gradients of any function (Section 2.1), so the TRI variants return
 * OFM_E_UNSUPPORTED.  X, grad: N x k device arrays of the workspace precision
 * (grad may be NULL); f_out: one FP64 in device memory.  Asynchronous; uses
 * the workspace's product buffers (call it between iterations, not inside).
 */
ofm_status ofm_objective(ofm_workspace ws, const void* X, double* f_out, void* grad,
                         hipStream_t stream);

/*
 * Per-pass device timing with HIP events recorded on the caller's stream
 * around the kernels of the selected passes (off by default).  Each pair of
 * events adds a few microseconds of host time and a short gap on the stream,
 * so time only the passes of interest inside a measured loop.
 * Pass ids (OFM_PASS_*) index host_ms / host_count; pass_mask bit i selects
 * pass i, 0 turns timing off, OFM_TIMING_ALL selects every pass.
 */
#define OFM_PASS_SPMM_X 0     /* A X with the fused direction epilogue        */
#define OFM_PASS_G 1          /* direction from a stored A X (recurrence; f2
                                 steps whose X^T A X is not yet known)        */
#define OFM_PASS_V 2          /* V = -G + V_prev diag(beta) and its products  */
#define OFM_PASS_SPMM_V 3     /* A V with the line-search products            */
#define OFM_PASS_LINESEARCH 4 /* cubic coefficients, roots, step sizes        */
#define OFM_PASS_UPDATE 5     /* X += V diag(alpha) and X^T X                 */
#define OFM_PASS_REDUCE 6     /* cross-block reductions of the k x k products */
#define OFM_PASS_RESIDUAL 7   /* residual and objective                       */
/* OFM_PASS_OTHER: products of set-up calls, and the f2 products X^T A V and
   V^T A V formed from a stored A V (k >= 32, without the recurrence) */
#define OFM_PASS_OTHER 8
#define OFM_NUM_PASSES 9
#define OFM_TIMING_ALL ((1u << OFM_NUM_PASSES) - 1u)
ofm_status ofm_set_timing(ofm_workspace ws, unsigned pass_mask);
/* Synchronizing: waits for the recorded events, adds the elapsed times (ms)
 * and launch counts since the last reset into host_ms[OFM_NUM_PASSES] and
 * host_count[OFM_NUM_PASSES]; reset != 0 clears the totals afterwards.  The
 * event pairs of timed launches are held (and their events not reused) until
 * this call, so a long timed run should call it from time to time. */
ofm_status ofm_get_timing(ofm_workspace ws, double* host_ms, int64_t* host_count, int reset);

/*
 * Y = scale[0] * X elementwise over count values of the given precision
 * (OFM_FP32 / OFM_FP64); scale is one FP64 in device memory; X == Y is
 * allowed.  The chain rule of the differentiable objectives: the gradient of
 * eqs. gradientf1 / gradientf2 (from ofm_objective) times the derivative that
 * arrives from the caller's loss, without a host synchronization.
 */
ofm_status ofm_scale(int64_t count, int precision, const double* scale, const void* X, void* Y,
                     hipStream_t stream);

/*
 * Algorithm 1, step 4: Y_l = X_l / ||X_l||_2 for every row (a zero row stays
 * zero).  X and Y are N x k of the given precision; X == Y is allowed.
 */
ofm_status ofm_row_normalize(int64_t n, int k, int precision, const void* X, void* Y,
                             hipStream_t stream);

/*
 * Algorithm 1, step 5, assignment step of Euclidean K-means:
 *   labels[l] = argmin_c sum_d (Y_ld - mu_cd)^2, lowest c on ties,
 *   dist2[l] = that minimum (nullable).
 * Y FP32 [n x dim], centroids FP32 [n_clusters x dim], dim in [1, 64],
 * n_clusters in [1, 1024].  Distances are accumulated in FP32.
 */
ofm_status ofm_kmeans_assign(int64_t n, int dim, int n_clusters, const float* Y,
                             const float* centroids, int32_t* labels, float* dist2,
                             hipStream_t stream);

/*
 * Euclidean K-means on the rows of Y (FP32 [n x dim]): k-means++ seeding
 * (Arthur & Vassilvitskii 2007) driven by the caller's uniforms
 * host_uniforms[0..n_clusters-1] in [0, 1) (centre 0 = point floor(u_0 n);
 * centre c = first point whose running sum of squared distances to the
 * nearest chosen centre exceeds u_c times the total), then Lloyd iterations
 * until no label changes or max_iter; an empty cluster keeps its centroid.
 * labels int32[n] and centroids FP32[n_clusters x dim] are outputs;
 * host_iters (nullable) receives the number of Lloyd iterations.
 * Synchronizing; allocates temporary device memory.
 */
ofm_status ofm_kmeans(int64_t n, int dim, int n_clusters, const float* Y,
                      const double* host_uniforms, int max_iter, int32_t* labels,
                      float* centroids, int32_t* host_iters, hipStream_t stream);

/*
 * ofm_kmeans without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, same kernels and bitwise the same results as
 * ofm_kmeans; its temporary buffers (squared distances and previous labels,
 * 8 bytes per point, the block partial sums of the centroids and a few small
 * arrays: ofm_kmeans_static_bytes(n, dim, n_clusters) bytes) live in one
 * file-scope device array of OFM_KMEANS_STATIC_BYTES (64 MiB) that every device
 * the library runs on holds until the process ends.  Calls on one device share
 * that array, so calls that overlap on one device (several host threads or
 * streams) race and must be serialized by the caller; each call initializes
 * what it reads.  Synchronizing.
 * Errors: as ofm_kmeans; OFM_E_SHAPE when the buffers of the call would exceed
 * OFM_KMEANS_STATIC_BYTES (e.g. n above about 7 million points at dim = 32
 * and 32 clusters).
 */
#define OFM_KMEANS_STATIC_BYTES ((size_t)64 << 20)
size_t ofm_kmeans_static_bytes(int64_t n, int dim, int n_clusters);
ofm_status ofm_kmeans_noalloc(int64_t n, int dim, int n_clusters, const float* Y,
                              const double* host_uniforms, int max_iter, int32_t* labels,
                              float* centroids, int32_t* host_iters, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* OFM_H */
