/*
 * spchol.h -- C ABI of the MI355X sparse Cholesky library (libspchol.so).
 *
 * The library factors symmetric positive definite matrices A whose sparsity
 * pattern is fixed while the values change, and solves A x = b with the
 * factor.  This is the setting the paper targets (Sec. 3.3: control flow
 * fixed by the input structure, cost amortized over many runs, few distinct
 * expression shapes): a one-time symbolic pass over the pattern plays the
 * role of the paper's expression-graph unrolling, decomposition and
 * grouping (Sec. 3.2, 4.2, 4.3), and each numeric call replays the grouped
 * work on the GPU.
 *
 * What is computed (textbook sparse Cholesky; the paper does not define it):
 *   A^ = P A P^T with A^_ij = A_{perm[i], perm[j]},  A^ = L L^T,
 *   x  = P^T L^{-T} L^{-1} P b.
 *
 * Conventions for every entry point
 *   - Every function returns an sc_status; no C++ exception crosses the ABI.
 *   - Pattern input: the lower triangle (diagonal included) in CSC form,
 *     colptr int64[n+1], rowind int32[nnz], rows strictly ascending inside a
 *     column and the diagonal first.  Anything else is SC_EPATTERN.
 *   - Values: float64, one value per stored pattern entry, in pattern order.
 *     Each off-diagonal value stands for both A_ij and A_ji.
 *   - perm (nullable = identity): int32[n], new index k <- old perm[k].
 *   - Pointers named *_host are host memory, *_dev device memory.  The
 *     caller owns them; the library only borrows them for the call (and,
 *     for asynchronous calls, until the stream reaches that point).
 *   - stream is a hipStream_t passed as void* (NULL = default stream).
 *     Numeric calls are asynchronous on that stream.
 *   - A plan is immutable after sc_analyze and may be shared by threads and
 *     streams.  A numeric object holds one batch of factors; calls that use
 *     the same numeric object must be ordered by the caller (same stream).
 */
#ifndef SPCHOL_H
#define SPCHOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SC_OK = 0,
    SC_EINVAL = -1,   /* bad argument (NULL, size, dtype, batch index ...) */
    SC_EPATTERN = -2, /* malformed pattern or permutation                  */
    SC_ENOMEM = -3,   /* host or device allocation failed                   */
    SC_EDEVICE = -4,  /* a HIP runtime call failed                          */
    SC_ENOTSPD = -5,  /* some matrix of the batch has a non-positive pivot  */
    SC_ENOCONV = -6,  /* iterative refinement did not meet its tolerance    */
    SC_ESCRATCH = -7  /* sc_solve_noalloc: the solve needs more workspace
                         than the static scratch holds                      */
} sc_status;

typedef enum { SC_F64 = 0, SC_F32 = 1 } sc_dtype;

typedef struct sc_plan sc_plan_t;       /* symbolic analysis (host + device) */
typedef struct sc_numeric sc_numeric_t; /* numeric factors of one batch      */

/* Options of the symbolic pass.  Fill with sc_options_default first. */
typedef struct {
    int32_t relax;        /* 1: merge a supernode into its parent when the
                             columns are contiguous and few explicit zeros
                             are added (default); 0: fundamental only     */
    int32_t relax_cols;   /* always merge while the merged width <= this  */
    double relax_zeros;   /* otherwise merge while the fraction of stored
                             zeros of the merged block stays below this   */
    int32_t small_front;  /* fronts with at most this many rows run in one
                             workgroup (up to 256 rows, and only if the
                             front fits the workgroup's LDS in FP64);
                             larger ones use the tiled kernels
                             (0 = library default)                         */
    int32_t soa_min_batch; /* numeric objects with at least this many
                             matrices solve in the batch-interleaved layout
                             (one matrix per lane; L is copied once per
                             factorization); 0 = library default (64, a
                             whole group of lanes), a negative value never */
    int32_t soa_seg_max;   /* in the batch-interleaved layout, a level whose
                             supernodes outside the panel kernels, times the
                             groups of 64 matrices, number at most this is
                             solved by the kernels that put one lane on each
                             row of a supernode instead (the top levels,
                             where one lane per matrix leaves the chip
                             idle); 0 = library default (96), a negative
                             value never */
    int32_t soa_subtree_min; /* in the batch-interleaved layout, the lowest
                             levels are solved as whole subtrees, one wave
                             per (subtree, group of 64 matrices), up to the
                             highest level that still has at least this
                             many such waves; 0 = library default (2048),
                             a negative value never (level by level)     */
    int32_t ordering;      /* elimination order: SC_ORDER_NATURAL, or
                             SC_ORDER_GIVEN (default: the caller's perm,
                             natural when perm is NULL), or SC_ORDER_ND
                             (built-in nested dissection of the pattern's
                             graph: separators from breadth-first level
                             structures rooted at pseudo-peripheral
                             vertices; perm must be NULL)                  */
    int32_t panel_inverse; /* batched solves (at least 16 matrices) of the
                             levels whose supernodes are solved by 64-column
                             panels, all at most 1024 columns wide: each
                             factorization also forms X = L11^{-1} of those
                             supernodes' diagonal blocks, and the solves
                             multiply by X (many workgroups per supernode)
                             instead of substituting panel after panel; the
                             results agree to rounding, not bit for bit.
                             0 = library default (on for SC_F32 factors, off
                             for SC_F64), 1 = on for both, a negative value
                             never                                          */
} sc_options;

/* Values of sc_options.ordering. */
enum { SC_ORDER_NATURAL = 0, SC_ORDER_GIVEN = 1, SC_ORDER_ND = 2 };

/* Sizes of a plan (per matrix of a batch). */
typedef struct {
    int64_t n;          /* order                                          */
    int64_t nnzA;       /* stored entries of the lower triangle of A      */
    int64_t nnzL;       /* structural nonzeros of L (exact pattern)       */
    int64_t nfund;      /* fundamental supernodes                         */
    int64_t nsuper;     /* supernodes after amalgamation                  */
    int64_t nlevels;    /* levels of the supernodal elimination tree      */
    int64_t L_store;    /* scalars of supernodal L storage (with padding) */
    int64_t U_store;    /* scalars of update-matrix workspace             */
    int64_t max_front;  /* largest front (rows)                           */
    int64_t max_width;  /* widest supernode (columns)                     */
    double flops;       /* sum_j c_j^2 over the exact column counts c_j   */
    int64_t etree_height; /* height of the column elimination tree        */
    int64_t nblocks;    /* independent diagonal blocks: the patterns of a
                           group plan, 1 for a plan from sc_analyze        */
} sc_plan_stats;

/* Human-readable name of a status code (static string). */
const char *sc_status_string(sc_status s);

/* Default options. */
sc_status sc_options_default(sc_options *opt);

/*
 * Symbolic analysis of the pattern (host only, no GPU work): validation,
 * permutation, elimination tree, column counts, fundamental and relaxed
 * supernodes, supernodal tree levels (longest path from the leaves, so
 * every dependency sits at a strictly lower level), relative index maps
 * and the value scatter map.  The plan copies what it needs; the inputs
 * may be freed after the call.  Device copies are made on first use.
 * The permutation used (given or computed) is reported by
 * sc_plan_export_symbolic.
 * Errors: SC_EINVAL (NULL pointers, n < 1, an ordering other than
 * SC_ORDER_GIVEN with a perm), SC_EPATTERN (unsorted or duplicate rows, a
 * row below the diagonal missing or out of range, missing or misplaced
 * diagonal, colptr not monotone, perm not a permutation), SC_ENOMEM.
 */
sc_status sc_analyze(int64_t n, const int64_t *colptr_host,
                     const int32_t *rowind_host, const int32_t *perm_host,
                     const sc_options *opt, sc_plan_t **plan_out);

/*
 * Group plan for an uneven batch: npat patterns (sizes n[k], lower CSC
 * colptr_host[k], rowind_host[k], optional perm_host[k], each with the
 * conventions above) analysed as the one block-diagonal matrix
 * diag(A_0, ..., A_{npat-1}), so that every level of every pattern runs in
 * the same launches (the paper's grouping of independent work, Sec. 4.3).
 * Layout of the group: pattern k owns columns [col0_k, col0_k + n[k]) and
 * values [val0_k, val0_k + nnz_k), concatenated in pattern order
 * (sc_plan_export_blocks gives the offsets); a value set of the group is
 * the concatenation of one value set of every pattern, a right-hand side
 * the concatenation of one vector of every pattern.  sc_factor_info and
 * sc_refine_solve report every pattern of every batch element on its own.
 * perm_host may be NULL (all natural) or have NULL entries.
 * Errors: as sc_analyze (checked per pattern), SC_EINVAL for npat < 1.
 */
sc_status sc_analyze_group(int32_t npat, const int64_t *n_host,
                           const int64_t *const *colptr_host,
                           const int32_t *const *rowind_host,
                           const int32_t *const *perm_host, const sc_options *opt,
                           sc_plan_t **plan_out);

sc_status sc_plan_info(const sc_plan_t *plan, sc_plan_stats *out);

/*
 * Block offsets of a plan (host memory, nblocks + 1 entries each, either
 * pointer may be NULL): col0_host[k] first column of block k (same in the
 * original and permuted numbering), val0_host[k] first value index.
 */
sc_status sc_plan_export_blocks(const sc_plan_t *plan, int64_t *col0_host,
                                int64_t *val0_host);

/*
 * Exact symbolic result in the permuted numbering, for checking: perm[n],
 * parent[n] (column elimination tree, -1 for roots), Lcolptr[n+1] and
 * Lrowind[nnzL] (row indices of every column of L ascending, diagonal
 * first; the pattern is structural and excludes amalgamation padding).
 * Any output pointer may be NULL.  All host memory.
 */
sc_status sc_plan_export_symbolic(const sc_plan_t *plan, int32_t *perm_host,
                                  int32_t *parent_host, int64_t *Lcolptr_host,
                                  int32_t *Lrowind_host);

/*
 * Supernode partition after amalgamation, for checking (host memory, any
 * pointer may be NULL): first[nsuper+1] column ranges, parent[nsuper]
 * supernodal elimination tree (-1 for roots), level[nsuper] (longest path
 * from the leaves), rowptr[nsuper+1] and rows[rowptr[nsuper]]: the row
 * structure of each front, ascending, starting with its own columns and
 * including rows added by amalgamation.
 */
sc_status sc_plan_export_supernodes(const sc_plan_t *plan, int32_t *first_host,
                                    int32_t *parent_host, int32_t *level_host,
                                    int64_t *rowptr_host, int32_t *rows_host);

void sc_plan_destroy(sc_plan_t *plan);

/*
 * Allocate device storage for `batch` factors of the plan's pattern in the
 * given precision (SC_F64, or SC_F32: FP32 factor with FP32 accumulation),
 * and a private non-blocking stream with two events on the current device
 * (the factorization runs part of the trailing updates of large fronts
 * there, ordered against the caller's stream by those events; a call
 * still returns with all its work ordered on the caller's stream).  Objects
 * that solve in the batch-interleaved layout (batch >= soa_min_batch) get a
 * second such stream with two events: the factorization copies L to that
 * layout there, beside its top levels, and joins it before returning.
 * Batches of at least 16 with whole-block inverses (sc_options.panel_inverse)
 * also hold those inverses (w^2 scalars per inverted supernode and matrix).
 * Uploads the plan to the current device if not done yet.
 * Errors: SC_EINVAL, SC_ENOMEM, SC_EDEVICE.
 */
sc_status sc_numeric_create(const sc_plan_t *plan, int32_t batch,
                            sc_dtype dtype, sc_numeric_t **num_out);

void sc_numeric_destroy(sc_numeric_t *num);

/*
 * Numeric factorization of a batch of value sets (same pattern):
 * values_dev is float64 [batch][ldv] with ldv >= nnzA; set b is factored
 * into factor b of `num`.  Overwrites any earlier factor in `num`.
 * Asynchronous; a non-positive pivot does not stop the call -- query it
 * with sc_factor_info.  Matrices of a batch never affect each other.
 * Errors: SC_EINVAL, SC_EDEVICE.
 */
sc_status sc_factor(const sc_plan_t *plan, sc_numeric_t *num,
                    const double *values_dev, int64_t ldv, void *stream);

/*
 * Per-matrix breakdown flags, info_host[b * nblocks + k] for block k of
 * batch element b (nblocks = 1 unless the plan is a group plan): 0 if that
 * factor is complete, else the smallest 1-based elimination step of the
 * block (permuted numbering, counted from the block's first column) whose
 * pivot failed d > 0; the factor of that block beyond that step is
 * unspecified, the other blocks are unaffected.  Synchronizes the stream.
 * Returns SC_ENOTSPD if any entry != 0.
 */
sc_status sc_factor_info(const sc_numeric_t *num, int32_t *info_host,
                         void *stream);

/*
 * Solve A x = b for every matrix of the batch: b_dev is float64
 * [batch][nrhs][ldb] (ldb >= n, original numbering), overwritten by x.
 * The triangular solves run in the precision of the stored factor: FP64
 * factors in FP64; FP32 factors with FP32 vectors and arithmetic (b is
 * rounded to FP32 on entry and x widened on exit), the precision in which
 * mixed-precision iterative refinement forms its corrections.
 * Asynchronous.  Errors: SC_EINVAL, SC_ENOMEM, SC_EDEVICE.
 */
sc_status sc_solve(const sc_plan_t *plan, sc_numeric_t *num, double *b_dev,
                   int32_t nrhs, int64_t ldb, void *stream);

/*
 * sc_solve without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results (bit for bit) as
 * sc_solve on the same numeric object, but the solve vectors live in a
 * static device array of SC_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on every GPU it runs on until the process ends, instead of the
 * numeric object's workspaces; the call makes no hipMalloc or hipFree and
 * calls no allocating routine.  The numeric object must come from
 * sc_numeric_create on the current device (which sets the device up).
 * Workspace need: 8 bytes x (matrices, rounded up to 64 in the
 * batch-interleaved layout) x nrhs x (n + the plan's front rows + the
 * panel partial sums), each of four vectors rounded up to 256 bytes.
 * Every call on one GPU shares that GPU's array, and the array keeps the
 * last call's contents (nothing in it needs to start at zero): calls that
 * overlap on one GPU (other streams, other threads, other numeric objects)
 * race, so the caller orders them.  Asynchronous on `stream`.
 * Errors: SC_EINVAL, SC_ESCRATCH (the workspace would exceed the array;
 * nothing is launched), SC_EDEVICE.
 */
#define SC_NOALLOC_SCRATCH_BYTES (32u << 20)
sc_status sc_solve_noalloc(const sc_plan_t *plan, sc_numeric_t *num, double *b_dev,
                           int32_t nrhs, int64_t ldb, void *stream);

/* Outcome of sc_refine_solve for one system: one (matrix, right-hand side,
   block) with block = the pattern of a group plan. */
typedef struct {
    int32_t iters;   /* corrections applied                               */
    int32_t clause;  /* 1: relres <= tol; 2: ||r||_2 <= 2 u ||A||_inf
                        ||x||_2 (FP64 evaluation floor, u = 2^-53);
                        0: neither after maxit corrections                */
    double relres;   /* ||b - A x||_2 / ||b||_2 at exit                   */
    double rnorm;    /* ||b - A x||_2                                     */
    double bnorm;    /* ||b||_2                                           */
    double xnorm;    /* ||x||_2                                           */
} sc_refine_stats;

/* Refinement methods of sc_refine_solve. */
enum { SC_REFINE_CLASSICAL = 0, SC_REFINE_PCG = 1 };

/*
 * Solve A x = b by iterative refinement with the factor in `num` (FP32 or
 * FP64) as the approximate inverse M^{-1}.  Both methods start from
 * x = solve(b) and run every vector operation in FP64 (A from values_dev,
 * the same values that were factored; solves use FP64 arithmetic on the
 * stored factor).
 *   SC_REFINE_CLASSICAL: while some system fails the stop rule and fewer
 *     than maxit corrections were applied: r = b - A x, x += solve(r).
 *   SC_REFINE_PCG: conjugate gradients on A preconditioned by the factor,
 *     at most maxit steps; the stop rule is tested on the true residual
 *     b - A x after each step, before the next direction is formed, so
 *     the step that meets the rule costs no further solve.  Converges when
 *     the factor's precision is too low for classical refinement
 *     (kappa(A) u_factor > 1).
 * Stop rule per system (matrix b, right-hand side r, block k; norms over
 * the block's rows, ||A||_inf of the block):
 * ||r||_2 <= tol ||b||_2, or ||r||_2 <= 2 u ||A||_inf ||x||_2 (the residual
 * has reached what FP64 can resolve).  A system that passes takes no
 * further corrections and keeps its record.
 * b_dev: float64 [batch][nrhs][ldb] (unchanged); x_dev: same shape, output.
 * stats_host (nullable): [batch][nrhs][nblocks] outcomes.  Synchronizes the stream
 * once per refinement step.  Returns SC_ENOCONV if some system did not meet
 * the rule (x then holds the last iterate).  Errors: SC_EINVAL, SC_ENOMEM,
 * SC_EDEVICE.
 */
sc_status sc_refine_solve(const sc_plan_t *plan, sc_numeric_t *num,
                          const double *values_dev, int64_t ldv,
                          const double *b_dev, double *x_dev, int32_t nrhs,
                          int64_t ldb, double tol, int32_t maxit, int32_t method,
                          sc_refine_stats *stats_host, void *stream);

/*
 * Copy factor values of the exact pattern to the host, for checking:
 * for each requested column j (permuted numbering) the values of
 * L[:, j] on rows Lrowind[Lcolptr[j] .. Lcolptr[j+1]) are appended to
 * out_host, in that order, as float64.  Synchronizes the device.
 * Errors: SC_EINVAL (bad batch index or column), SC_EDEVICE.
 */
sc_status sc_numeric_get_columns(const sc_plan_t *plan,
                                 const sc_numeric_t *num, int32_t b,
                                 int64_t ncols, const int32_t *cols_host,
                                 double *out_host);

/*
 * Copy the whole stored block of supernode s of factor b to the host, for
 * checking: c x w scalars, column-major (c = rows of the front, w = its
 * columns, as sc_plan_export_supernodes gives them), as float64.  Rows of
 * column t of the block are the front's rows t .. c-1 (entries above the
 * diagonal, rows 0 .. t-1, hold no factor values).  Stored entries outside
 * the exact pattern of L (amalgamation padding) are included: they come
 * out as 0.0.  Synchronizes the device.
 * Errors: SC_EINVAL (bad batch index or supernode), SC_EDEVICE.
 */
sc_status sc_numeric_get_block(const sc_plan_t *plan, const sc_numeric_t *num, int32_t b,
                               int32_t s, double *out_host);

/* Per-kernel totals of timed launches (see sc_numeric_profile). */
typedef struct {
    char name[32];    /* kernel name                                      */
    int64_t launches; /* launches timed                                   */
    double ms;        /* summed event time of those launches              */
    double flops;     /* algorithmic flops of those launches              */
    double bytes;     /* the library's byte model of those launches: front
                         and update blocks, vectors and indices moved     */
    double alg_bytes; /* algorithmic bytes of the method: factor launches
                         the entries of A read (12 B: value and row index)
                         plus the exact entries of L written; triangular
                         solves the exact entries of L read once for all
                         right-hand sides; residual products the entries of
                         A read (12 B); other launches 0                  */
} sc_kernel_stat;

/*
 * Measurement support: with enable != 0, every later launch made for this
 * numeric object (factor and solve) is bracketed by two HIP events on the
 * stream it runs on, and its algorithmic flops and bytes are recorded;
 * enable = 0 stops recording.  Timing adds two event records per launch.
 */
sc_status sc_numeric_profile(sc_numeric_t *num, int32_t enable);

/*
 * Wait for the recorded launches, sum them per kernel into out_host (at
 * most cap entries; *count_out receives the number written) and clear the
 * record.  Errors: SC_EINVAL, SC_EDEVICE.
 */
sc_status sc_numeric_profile_read(sc_numeric_t *num, int32_t cap,
                                  sc_kernel_stat *out_host,
                                  int32_t *count_out);

/*
 * Adjoint of the solve (gradients of a loss L(x) through x = A^{-1} b, the
 * closed form of differentiating the solve; the paper differentiates its
 * unrolled expression graph symbolically, Sec. 4.9): with the factor of
 * the last sc_factor on this numeric object,
 *     lambda = A^{-1} g_x                      -> gb_dev (dL/db)
 *     dL/dv_k = -sum_r (lambda_i x_j + lambda_j x_i)   stored entry (i, j), i > j
 *     dL/dv_k = -sum_r lambda_i x_i                    diagonal entry
 *                                              -> gvalues_dev [batch][ldv]
 * x_dev, gx_dev and gb_dev are [batch][nrhs][ldb] float64 (device), x the
 * solution of the forward solve, gx the upstream gradient dL/dx; gb_dev may
 * alias gx_dev (overwritten) but not x_dev.  The arithmetic is FP64; with an
 * FP32 factor lambda carries the factor's accuracy.  One extra solve plus
 * one pass over the stored entries; asynchronous on `stream`.  Errors:
 * SC_EINVAL, SC_ENOMEM, SC_EDEVICE.
 */
sc_status sc_adjoint(const sc_plan_t *plan, sc_numeric_t *num, const double *x_dev,
                     const double *gx_dev, double *gvalues_dev, int64_t ldv, double *gb_dev,
                     int32_t nrhs, int64_t ldb, void *stream);

/*
 * One captured step for repeated use on fixed buffers (the paper's setting:
 * the same structure run many times, Sec. 3.3): the factorization of the
 * whole batch from values_dev (as sc_factor) followed by the refined solve
 * b_dev -> x_dev (as sc_refine_solve with maxit = iters), recorded once into
 * a HIP graph and replayed by sc_step_graph_launch.  The replay runs exactly
 * `iters` refinement steps with no host synchronization: a system that has
 * met the stop rule is skipped on the device from then on, so the result of
 * every system equals the one of sc_refine_solve with the same maxit.
 * Creation allocates every workspace and captures on a private stream; the
 * numeric object, values_dev, b_dev and x_dev must stay valid and unmoved
 * while the graph exists, and the numeric object must not be used by other
 * calls while a replay is in flight.  The graph holds the addresses of the
 * numeric object's workspaces: while any graph of the object exists, a call
 * on it that would need larger workspaces (sc_solve, sc_refine_solve,
 * sc_adjoint or another sc_step_graph_create with more right-hand sides or
 * a larger ldb) returns SC_EINVAL instead of reallocating them.  Destroy
 * the graphs before the numeric object.  Errors: SC_EINVAL (bad argument, or
 * b_dev == x_dev), SC_ENOMEM, SC_EDEVICE.
 */
typedef struct sc_graph sc_graph_t;
sc_status sc_step_graph_create(const sc_plan_t *plan, sc_numeric_t *num,
                               const double *values_dev, int64_t ldv,
                               const double *b_dev, double *x_dev, int32_t nrhs,
                               int64_t ldb, double tol, int32_t iters, int32_t method,
                               sc_graph_t **graph_out);
/* Replay the step on `stream` (asynchronous). */
sc_status sc_step_graph_launch(sc_graph_t *graph, void *stream);
/* Per-system refinement statistics of the last replay, as in
 * sc_refine_solve (synchronizes `stream`); SC_ENOCONV if a system has not
 * met the stop rule. */
sc_status sc_step_graph_stats(sc_graph_t *graph, sc_refine_stats *stats_host, void *stream);
void sc_step_graph_destroy(sc_graph_t *graph);

/*
 * Autotuner (grouping, kernel thresholds and solve layout of a workload):
 * for each candidate option set (fronts handled in one workgroup up to 32,
 * 64 or 128 rows; amalgamation width 4 or 16; for batches of at least 16
 * the row-major or the batch-interleaved solve) it analyzes the pattern,
 * factors the caller's batch and solves the caller's right-hand sides on
 * `stream`, timed with HIP events (best of two after a warm-up), and
 * returns in best_out the set with the smallest
 *     factor_ms + solves_per_factor * solve_ms.
 * Pattern arguments as in sc_analyze (host), values_dev [batch][ldv] and
 * b_dev [batch][nrhs][ldb] on the device (b_dev is not modified; the
 * library allocates a scratch copy).  When perm_host is NULL the
 * candidates are also tried with the natural and the built-in nested
 * dissection orderings (best_out->ordering reports the choice); a given
 * permutation is always kept.  table_host (nullable when
 * table_cap == 0) receives up to table_cap measured candidates and
 * *ntable_out their number.  Synchronizes `stream`.  Errors: SC_EINVAL,
 * SC_EPATTERN, SC_ENOMEM, SC_EDEVICE, SC_ENOTSPD is not reported (info is
 * the caller's to check on the chosen plan).
 */
typedef struct {
    sc_options opt;   /* the candidate                                   */
    double factor_ms; /* factorization of the batch                      */
    double solve_ms;  /* one solve of every right-hand side              */
    double score;     /* factor_ms + solves_per_factor * solve_ms        */
} sc_tune_entry;
sc_status sc_autotune(int64_t n, const int64_t *colptr_host, const int32_t *rowind_host,
                      const int32_t *perm_host, const double *values_dev, int64_t ldv,
                      int32_t batch, sc_dtype dtype, const double *b_dev, int32_t nrhs,
                      int64_t ldb, double solves_per_factor, sc_options *best_out,
                      sc_tune_entry *table_host, int32_t table_cap, int32_t *ntable_out,
                      void *stream);

/*
 * The autotuner for an uneven batch: the same candidates and score as
 * sc_autotune, each analysed as the group plan of sc_analyze_group (pattern
 * arguments as there, host memory) and timed on the caller's concatenated
 * value sets and right-hand sides (values_dev [batch][ldv], b_dev
 * [batch][nrhs][ldb] with ldb >= the group's order).  Errors as
 * sc_autotune.
 */
sc_status sc_autotune_group(int32_t npat, const int64_t *n_host,
                            const int64_t *const *colptr_host, const int32_t *const *rowind_host,
                            const int32_t *const *perm_host, const double *values_dev,
                            int64_t ldv, int32_t batch, sc_dtype dtype, const double *b_dev,
                            int32_t nrhs, int64_t ldb, double solves_per_factor,
                            sc_options *best_out, sc_tune_entry *table_host, int32_t table_cap,
                            int32_t *ntable_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPCHOL_H */
