/*
 * cktlu -- circuit sparse LU for MI355X (gfx950): the C ABI.
 *
 * The library follows the solver structure of CKTSO (Chen, "CKTSO:
 * High-Performance Parallel Sparse Linear Solver for General Circuit
 * Simulations", IEEE TCAD): a one-time pre-processing step, a numerical
 * factorization in every Newton-Raphson iteration, and triangular solves
 * (Section III, Fig. 4).  Matrices are CSC and factored left-looking, which is
 * the paper's up-looking row algorithm applied to the transpose (Section II-A).
 *
 * Conventions for every entry point:
 *   - return value: 0 = success, > 0 = success with a warning (CKTLU_W_*),
 *     < 0 = error (CKTLU_E_*); cktlu_strerror() names each code;
 *   - integer arrays are int32, 0-based; CSC inputs have sorted row indices
 *     inside each column and no duplicates;
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *     device memory of the current device (e.g. a PyTorch CUDA tensor);
 *   - the caller owns every pointer it passes and keeps device buffers alive
 *     until the work queued on the context's stream has completed; the library
 *     copies the host pattern arrays it needs and owns the device memory it
 *     allocates (patterns, factors, schedules), released by cktlu_destroy();
 *   - one context per circuit; all device work of a context is ordered on its
 *     stream; a context is not safe for concurrent calls from several threads.
 *   - call order: create -> analyze -> factorize[_host] -> (refactorize ->
 *     solve)*; a call out of order returns CKTLU_E_STATE.
 */
#ifndef CKTLU_H
#define CKTLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CKTLU_OK 0
#define CKTLU_W_REPIVOTED 1     /* a pivot check failed; the fallback re-pivoted (pattern may change) */
#define CKTLU_W_IR_FALLBACK 2   /* FP32 refinement did not reach the tolerance; FP64 path used */
#define CKTLU_E_ARG (-1)        /* invalid argument (bad CSC, bad size, NULL pointer) */
#define CKTLU_E_STATE (-2)      /* call out of order */
#define CKTLU_E_STRUCT_SINGULAR (-3) /* no zero-free diagonal exists / empty candidate set */
#define CKTLU_E_NUM_SINGULAR (-4)    /* zero or non-finite pivot after pivoting */
#define CKTLU_E_NOMEM (-5)      /* host or device allocation failed */
#define CKTLU_E_HIP (-6)        /* a HIP runtime call failed */
#define CKTLU_E_LIMIT (-7)      /* a size exceeds a documented limit */

/* precision of the factors */
#define CKTLU_FP64 0            /* FP64 factors and solves */
#define CKTLU_FP32_IR 1         /* FP32 factors, FP64 residual / update / pivot test, iterative refinement */

/* fill-reducing ordering used by analyze */
#define CKTLU_ORDER_AMD 0       /* approximate minimum degree on the pattern of B + B' */
#define CKTLU_ORDER_NATURAL 1   /* keep the (transversal-permuted) natural order */
#define CKTLU_ORDER_AMF 2       /* approximate minimum fill on the pattern of B + B' */
#define CKTLU_ORDER_AUTO 3      /* AMD, AMF, ND and ND + constrained AMD; keep the one whose symbolic Cholesky of
                                   B + B' has the fewest entries (ties: the earlier), the combined ordering of
                                   Section III-A */
#define CKTLU_ORDER_ND 4        /* nested dissection (level-set separators), AMD on parts of <= 4096 nodes */
#define CKTLU_ORDER_ND_CAMD 5   /* the same dissection stopped at its parts, then one constrained minimum degree
                                   over the whole pattern that eliminates the parts in the dissection's order
                                   (Section III-A) */

typedef struct cktlu_ctx cktlu_ctx;

typedef struct {
    double pivot_eps;      /* threshold eps of the pivot rule (Section II-A); default 1e-3, range (0, 1] */
    int precision;         /* CKTLU_FP64 (default) or CKTLU_FP32_IR */
    double ir_tol;         /* FP32_IR: backward-error target; default 1e-10 */
    int ir_max_iter;       /* FP32_IR: refinement step limit; default 10 */
    int ordering;          /* CKTLU_ORDER_*; default AUTO (AMD, AMF and ND, the one with the least fill) */
    int transversal;       /* 1 (default): structural maximum transversal before ordering */
    void *stream;          /* hipStream_t for all device work; NULL = the null stream */
    int force_fail_col;    /* test hook: >= 0 makes the pivot check of this column fail once */
    int dense_tail_size;   /* schedule: order D of the trailing block factored densely (Section V-A);
                              0 = automatic (largest multiple of 64 in [256, 8192] whose block of L+U
                              reaches dense_tail_density), -1 = never, > 0 = exactly min(value, n) */
    double dense_tail_density; /* schedule: minimum fill density for the automatic choice; default 0.3 */
    int timing;            /* 1: record HIP events around each device phase (read by cktlu_get_timing) */
    int solve_chain_width; /* solves: consecutive levels of the solve graphs with at most this many rows run
                              in one launch, one workgroup per instance stepping through them; 0 = automatic
                              (currently one launch per level: chained levels run their rows one after another
                              on one CU, which measured slower on long rows), -1 = one launch per level */
    int dense_panel_width; /* dense block: columns factored between two updates of the whole trailing block
                              (64, 128 or 256; panels of 64 inside update only the rest of their group);
                              0 = automatic (256) */
    int dense_lookahead;   /* dense block: 1 runs the panels of the next group on a second stream of the
                              context while the trailing update of the current group runs (same results);
                              0 (default) = one stream, which measured faster: the update's workgroups fill
                              the device and the panels waited for them */
    int dense_device_repivot; /* pivot-check fallback: 0 (default) re-factors the dense block on the device
                              with the threshold pivot rule when every column to restart lies in it (the
                              host then computes only the new pattern); -1 = always the host fallback */
    int sweep_slot_map;    /* 0 (default): the schedule (built by the factorizations) records, for every
                              entry of every update task's sources, its slot in the target column: 4 bytes
                              per multiply-add of the sweep, built on the host only when a device is present
                              and the map takes at most a quarter of its free HBM (autotuner trials: at most
                              2^30 entries).  The sweep then loads the slot instead of searching the target's
                              rows; results are bit-identical.  -1 = never */
    int sweep_supernodes;  /* 0 (default): the sweep runs on supernodes of up to 64 columns (runs of columns
                              with a dense diagonal block and shared rows below it): per dependency level of
                              the supernodes, one launch factors their diagonal blocks and panels densely and
                              one applies them to their target columns; -1: the column sweep (one launch per
                              right-looking level of single columns, with the slot map above) */
    int static_pivoting;   /* pre-processing with values (cktlu_analyze_values; Section III-A): 0 (default) the
                              structural transversal only; 1 the row permutation P that maximises the product
                              of the diagonal magnitudes (maximum-weight matching); 2 that P and scalings S_r,
                              S_c with |diagonal| = 1 and every other entry at most 1 in magnitude: the library
                              then factors S_r P A S_c (its factors, pivot tests and getters refer to that
                              matrix) while values, right-hand sides and solutions stay the caller's */
    int sweep_panel_rows;  /* supernodal sweep: a panel with more rows below its diagonal block than this is
                              split into units of about this many rows (a workgroup each; panels of at most
                              16 columns: half as many rows, a wavefront each), whose column maxima meet
                              for the pivot test; 0 = 256, else 16 .. 65536.  Same results for any value */
    int solve_split_entries; /* supernodal solves: a supernode pulls its entries outside the diagonal block
                              as runs (a column and the consecutive rows of the supernode in it), split into
                              units (a workgroup each) whose partial sums are added in a fixed order; a
                              level's units hold its runs / 128, clamped to solve_split_entries / 64 ..
                              solve_split_entries / 16 runs; 0 = 8192, else 64 .. 2^30.  Sums are grouped
                              differently per value (rounding only) */
} cktlu_options;

typedef struct {
    int repivoted;         /* 1 if a pivot check failed and the fallback ran */
    int first_fail_col;    /* smallest column whose check failed, -1 if none */
    int restart_size;      /* columns recomputed with pivoting by the fallback */
    int pattern_changed;   /* 1 if the factor pattern changed (schedules rebuilt) */
} cktlu_refactor_info;

typedef struct {
    int ir_iters;          /* refinement steps taken (0 in FP64 mode) */
    double backward_err;   /* FP32_IR: final eta_inf of the first right-hand side; FP64: -1 (not computed) */
    int used_fp64;         /* 1 if the FP32_IR solve fell back to FP64 factors */
} cktlu_solve_info;

typedef struct {
    int64_t n, nnz_a, nnz_l, nnz_u;   /* nnz_l: strictly lower L; nnz_u: U incl. diagonal */
    double flops;                     /* factorization FLOPs: 2*MACs + divisions (Section VI) */
    double macs;                      /* multiply-adds of the left-looking update */
    int64_t levels, max_width;        /* dependency-graph levels and widest level */
    int64_t etree_height;             /* height of the column elimination tree */
    int64_t dense_tail;               /* order of the trailing block factored densely (0 = none) */
    int64_t n_factorize, n_refactorize, n_repivot, n_restart_cols;
    int64_t n_fp64_fallback_solves;
    double bytes_refactor, bytes_solve;  /* algorithmic HBM bytes per refactorization / per RHS solve */
    double macs_sweep;                /* multiply-adds of the sparse sweep's update tasks */
    double bytes_sweep;               /* its traffic model, what the sweep moves when nothing is reused
                                         from caches: supernodal, 8 per panel or update multiply-add (L
                                         value) + 20 per row of R updated (slot, target read and written);
                                         column sweep, 28 per MAC (L value + row index gathered, target read
                                         and written); both + 24 per L entry of a sparse column (pivot test
                                         read, division read and write) */
    double flops_dense;               /* FLOPs of the dense trailing block's LU (2/3 D^3 + lower order) */
    double macs_schur;                /* multiply-adds of the dense block's update by the sparse columns */
    int64_t sweep_launches;           /* kernel launches of one sparse sweep */
    int64_t dense_launches;           /* kernel launches of one dense-block factorization */
    int64_t solve_launches;           /* kernel launches of one triangular solve pass (L and U) */
    int64_t n_device_repivot;         /* fallbacks whose restart set lay inside the dense block and were
                                         re-factored on the device (pivoted dense LU) */
    int64_t ordering_used;            /* CKTLU_ORDER_* that analyze applied */
    int64_t fill_amd, fill_amf, fill_nd;  /* CKTLU_ORDER_AUTO: entries of the symbolic Cholesky factor of
                                         B + B' under each method (-1 when not run) */
    int64_t slot_map_entries;         /* entries of the sweep's slot map on the device (0: none, the sweep
                                         searches the target rows) */
    int64_t schur_parts, schur_scratch_cols;  /* the dense block's Schur update: parts (wavefronts per
                                         instance) and scratch columns of the parts after a column's first */
    double entries_sweep;             /* factor entries the sweep finalises: every entry of the sparse
                                         columns and the dense columns' entries in sparse rows */
    double entries_dense;             /* factor entries of the dense columns in dense rows */
    double macs_dense;                /* multiply-adds of the dense block's own LU (the method's work inside
                                         it; the blocked dense LU issues 2/3 D^3 flops) */
    double alg_bytes_refactor_sweep;  /* compulsory bytes of the sweep: an index read and a value written per
                                         entry it finalises (12 bytes in FP64, 8 with FP32 factors) */
    int64_t sweep_supernodes;         /* supernodes of the supernodal sweep (0: the column sweep runs) */
    int64_t sweep_levels;             /* dependency levels of the sweep (supernodal or right-looking) */
    int64_t fill_ndc;                 /* CKTLU_ORDER_AUTO: the same count under ND + constrained AMD */
    int64_t n_fp32_check_retries;     /* FP32_IR refactorizations whose pivot test failed on the FP32 values
                                         and passed in FP64 (the context then keeps FP64 factors) */
} cktlu_stats;

/* Device time of the phases, accumulated over the calls made with options.timing = 1
 * (HIP events on the context's stream). */
typedef struct {
    double init_ms;        /* value scatter into the factor storage */
    double sweep_ms;       /* right-looking level sweep over the sparse columns */
    double dense_ms;       /* dense trailing block LU: panels, MFMA updates, pivot test, scatter */
    double solve_sparse_ms;/* sparse levels of the L and U solves */
    double solve_dense_ms; /* dense block solves */
    int64_t refactors;     /* refactorizations timed */
    int64_t solve_passes;  /* triangular solve passes timed (each covers up to 8 right-hand sides) */
    int64_t sweep_launches, dense_launches, solve_sparse_launches, solve_dense_launches;
    double schur_ms;       /* the sparse columns' update of the dense block, S -= L21 U12 (not in dense_ms) */
} cktlu_timing;

/* Fill *opt with defaults. */
void cktlu_default_options(cktlu_options *opt);

/* Create a context.  opt may be NULL (defaults).  *out is NULL on failure. */
int cktlu_create(cktlu_ctx **out, const cktlu_options *opt);

/* Release all host and device memory of the context.  NULL is ignored. */
void cktlu_destroy(cktlu_ctx *ctx);

/* Human-readable name of a status code (static string). */
const char *cktlu_strerror(int status);

/* Change the stream used for device work (hipStream_t, NULL = null stream). */
int cktlu_set_stream(cktlu_ctx *ctx, void *stream);

/*
 * Pre-processing (Section III-A), host only, once per pattern: validates the
 * CSC pattern (host, n x n, colptr[n+1], rowind[colptr[n]]), finds a
 * structural maximum transversal (a zero-free diagonal), computes the
 * fill-reducing symmetric ordering and the column elimination tree of the
 * permuted matrix (Section II-B).  Does not touch the device.
 * Errors: E_ARG, E_STRUCT_SINGULAR, E_NOMEM.
 */
int cktlu_analyze(cktlu_ctx *ctx, int32_t n, const int32_t *colptr, const int32_t *rowind);

/*
 * cktlu_analyze with the matrix values (host, nnz FP64 in the CSC order): with
 * options.static_pivoting = 1 or 2 the transversal is the maximum-product
 * matching of the values (and 2 computes the scaling), so that large entries
 * sit on the diagonal before the ordering (Section III-A); when the nonzero
 * values admit no perfect matching the structural transversal is used and no
 * scaling.  With static_pivoting = 0 it equals cktlu_analyze.  Errors: those
 * of cktlu_analyze, and E_ARG for NULL values with static_pivoting > 0.
 */
int cktlu_analyze_values(cktlu_ctx *ctx, int32_t n, const int32_t *colptr, const int32_t *rowind,
                         const double *values);

/* The static scaling of the last analyze (host out, double[n] each, either may be
 * NULL): the factored matrix is rscale[i] A(i, j) cscale[j] (all ones without
 * scaling).  Errors: E_ARG, E_STATE. */
int cktlu_get_scaling(const cktlu_ctx *ctx, double *rscale, double *cscale);

/*
 * Factorization with pivoting (Section II-A, Algorithm 1): threshold partial
 * pivoting on the host, then the dependency schedule (Section II-B) and the
 * device layout are built and uploaded.  values_dev: device, nnz FP64 values
 * in analyze()'s CSC order.  The preferred pivot of each column is the row in
 * its position under the previous pivot sequence (identity the first time).
 * Synchronises the context's stream.  Errors: E_STATE, E_STRUCT_SINGULAR,
 * E_NUM_SINGULAR, E_NOMEM, E_HIP.
 */
int cktlu_factorize(cktlu_ctx *ctx, const double *values_dev);

/* Same as cktlu_factorize with host values (no device work until the next
 * device call, which uploads the factors and these values: an FP32_IR solve
 * right after it refines against them).  Usable without a GPU. */
int cktlu_factorize_host(cktlu_ctx *ctx, const double *values_host);

/*
 * Fast factorization with pivot check (Section IV): the stored pattern and
 * pivot sequence are reused; every column is updated on the device in a
 * dependency-ordered schedule and its pivot is tested against eps times the
 * largest entry of its L part.  When a test fails, the remaining work stops,
 * the restart set (unfinished columns and their elimination-tree ancestors,
 * Section IV-C) is refactored with pivoting on the host (Section IV-D), the
 * schedule is rebuilt for the new pattern and CKTLU_W_REPIVOTED is returned.
 * values_dev: device, nnz FP64 values in analyze()'s CSC order.  info may be
 * NULL.  Synchronises the stream once (a 16-byte status read).
 * Errors: E_STATE, E_NUM_SINGULAR, E_NOMEM, E_HIP.
 */
int cktlu_refactorize(cktlu_ctx *ctx, const double *values_dev, cktlu_refactor_info *info);

/*
 * Re-factorization without pivot check (Section II-A, Algorithm 1 without its
 * symbolic and pivoting lines): the check-free counterpart of
 * cktlu_refactorize, kept to measure the cost of the check.  Never re-pivots.
 */
int cktlu_refactorize_nocheck(cktlu_ctx *ctx, const double *values_dev);

/*
 * Triangular solves (Section II-C, Algorithm 2; Section V): x = A^{-1} b for
 * nrhs right-hand sides.  b_dev: device, column r at b_dev + r*ldb (ldb >= n);
 * x_dev: device, column r at x_dev + r*ldx (ldx >= n); b and x must not
 * overlap.  In FP32_IR mode the residual, the update and the stopping test run
 * in FP64 against the values of the last refactorization (backward error
 * eta_inf <= ir_tol), falling back to FP64 factors when refinement stalls
 * (W_IR_FALLBACK); the first two refinement steps are queued together and
 * decide convergence on the device, so the host waits once for them.  After such a fallback the context keeps FP64 factors for
 * its refactorizations and solves (info->used_fp64 = 1) until the next
 * cktlu_factorize: a circuit too ill-conditioned for FP32 factors stays so
 * while its values move by NR steps.  The same holds after a refactorization
 * whose pivot test failed on the FP32 values but passed in FP64.  info may be NULL.  Errors: E_STATE,
 * E_ARG, E_HIP.
 */
int cktlu_solve(cktlu_ctx *ctx, int32_t nrhs, const double *b_dev, int32_t ldb,
                double *x_dev, int32_t ldx, cktlu_solve_info *info);

/*
 * The solve of cktlu_solve without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels and results as cktlu_solve, with the
 * work rows in a file-scope device array of the library instead of a buffer it
 * allocates.  The array holds 2^19 rows (64 MiB, one copy per GPU the library
 * runs on, kept until the process ends); every call on a GPU shares it, so
 * calls that overlap on one GPU (several streams or threads) race, and a call
 * writes every row it reads.  Requires FP64 factors already on the device
 * (after cktlu_factorize or cktlu_refactorize on a context in FP64 mode, or in
 * FP32_IR mode after a fallback to FP64 factors).  b_dev, x_dev, ldb, ldx as
 * in cktlu_solve.  Errors: E_ARG, E_STATE (no device factors, FP32 factors),
 * E_LIMIT (n > 2^19), E_HIP.
 */
int cktlu_solve_noalloc(cktlu_ctx *ctx, int32_t nrhs, const double *b_dev, int32_t ldb, double *x_dev,
                        int32_t ldx);

/*
 * Batched fast factorization of `batch` same-pattern instances (Monte-Carlo
 * corners).  values_dev: device, batch x nnz FP64 values, instance i at
 * values_dev + i*nnz.  status_dev: device int32[batch]; entry i is set to -1
 * when instance i passed every pivot check, else to its smallest failing
 * column.  No host synchronisation and no fallback; the factors stay resident
 * for cktlu_solve_batched.  Errors: E_STATE, E_ARG, E_NOMEM, E_HIP.
 */
int cktlu_refactorize_batched(cktlu_ctx *ctx, int32_t batch, const double *values_dev,
                              int32_t *status_dev);

/*
 * Solves with the resident factors of the last cktlu_refactorize_batched.
 * b_dev: device, batch x nrhs x n FP64 (instance i, rhs r at (i*nrhs + r)*n),
 * nrhs <= 8; x_dev: same layout.  status_dev: the status array of that call;
 * instances whose status is not -1 are skipped (their x is left unchanged).
 * FP32_IR mode: every instance is refined in FP64 (residual with its own
 * values) until eta_inf <= ir_tol; converged instances leave the refinement,
 * the host checks progress after each step (one synchronisation per step).
 * Instances that reach ir_max_iter or stall are re-solved with FP64 factors
 * of their values (all instances are re-factored in FP64 for that), and the
 * call returns W_IR_FALLBACK.  eta_dev (device, double[batch], may be NULL)
 * receives each instance's final eta_inf in FP32_IR mode (-1 if skipped or
 * in FP64 mode).  Errors: E_STATE, E_ARG, E_NOMEM, E_HIP.
 */
int cktlu_solve_batched(cktlu_ctx *ctx, int32_t batch, int32_t nrhs, const double *b_dev,
                        double *x_dev, const int32_t *status_dev, double *eta_dev);

/*
 * One Newton-Raphson step of many same-pattern instances (Monte-Carlo corners)
 * as a single captured HIP graph: the refactorization of cktlu_refactorize_batched
 * (status_dev as there) followed by the solve of cktlu_solve_batched for nrhs
 * right-hand sides (b_dev, x_dev as there).  FP64: a plain solve.  FP32_IR:
 * FP32 factors and exactly ir_steps FP64 refinement steps (>= 1) decided on the
 * device, each instance leaving once its eta_inf reaches ir_tol; eta_dev
 * (device, double[batch], may be NULL) receives each instance's last eta_inf
 * (-1 for instances that failed the pivot test, and in FP64 mode).  No host
 * synchronisation: the caller reads status and eta afterwards and handles the
 * instances that failed the pivot test or did not reach ir_tol (for instance
 * with cktlu_solve_batched).  The graph is captured on the first call and
 * replayed while batch, nrhs, ir_steps and every pointer stay the same and the
 * library's device buffers have not moved; otherwise it is captured again (the
 * capture synchronises the context's stream).  Errors: E_STATE, E_ARG, E_LIMIT,
 * E_NOMEM, E_HIP.
 */
int cktlu_step_batched_graph(cktlu_ctx *ctx, int32_t batch, const double *values_dev, int32_t *status_dev,
                             int32_t nrhs, const double *b_dev, double *x_dev, double *eta_dev,
                             int32_t ir_steps);

/* Result of cktlu_autotune. */
typedef struct {
    int32_t n_tried;              /* schedules measured */
    int32_t dense_tail[16];       /* order D of the dense trailing block of each (0 = none) */
    double ms_per_step[16];       /* device time of one refactorization + solve of `batch` instances */
    int32_t best;                 /* index of the fastest, now in use */
    /* second stage, with that D: the knobs the caller left at 0, one at a time */
    int32_t n_knob_tried;         /* trials of the second stage */
    int32_t knob[16];             /* CKTLU_KNOB_* of each trial */
    int32_t knob_value[16];       /* the value tried */
    double knob_ms_per_step[16];  /* its device time per step */
    int32_t sweep_supernodes, sweep_panel_rows, solve_split_entries, dense_panel_width;  /* kept (0 = default) */
} cktlu_tune_result;

#define CKTLU_KNOB_SUPERNODE_WIDTH 0   /* options.sweep_supernodes: 64 (default) or 32 columns */
#define CKTLU_KNOB_PANEL_ROWS 1        /* options.sweep_panel_rows: 256 (default), 128 or 512 */
#define CKTLU_KNOB_SOLVE_SPLIT 2       /* options.solve_split_entries: 8192 (default), 4096 or 16384 */
#define CKTLU_KNOB_DENSE_PANEL 3       /* options.dense_panel_width: 256 (default) or 128 */

/*
 * Schedule autotuner (the dense-part threshold the paper fixes for its CPUs,
 * Section V-A, chosen here by measurement on the device): for each candidate
 * order D of the dense trailing block (none, the density rule at 0.5, 0.3 and
 * 0.2, D = 512, 1024, 2048, 4096, 8192 up to n, and 10240, 12288, 16384 while
 * batch blocks of that order fit a quarter of the free device memory;
 * duplicates skipped) the
 * schedule is rebuilt and uploaded, and `reps` steps are timed with HIP events
 * on the context's stream, a step being the refactorization of `batch`
 * instances (values_dev: batch x nnz, as cktlu_refactorize_batched; batch 1
 * uses cktlu_refactorize) plus a solve of one right-hand side each.  The
 * fastest schedule stays in use (options.dense_tail_size is set to it).  A
 * second stage then tries, with that D and one knob at a time, the other
 * values of each schedule knob the caller left at 0 (CKTLU_KNOB_*: the paper's
 * CPU constants have GPU counterparts in the supernode width, the rows per
 * panel unit, the entries per solve unit and the dense panel width), keeping
 * a value when it is at least 2% faster.
 * The factors on the device are those of the last timed step.  Errors:
 * E_STATE, E_ARG, E_NOMEM, E_HIP.
 */
int cktlu_autotune(cktlu_ctx *ctx, int32_t batch, const double *values_dev, int32_t reps,
                   cktlu_tune_result *out);

/*
 * Restart set of the pivot-check fallback (Section IV-C), host only: in_set[k]
 * = 1 for every column k with unfinished[k] != 0 and for every ancestor of such
 * a column in the column elimination tree, 0 for the others.  parent: host
 * int32[n], the tree (-1 = root; every other entry satisfies k < parent[k] < n,
 * as cktlu_get_analysis returns it); unfinished, in_set: host int32[n].
 * Errors: E_ARG (NULL pointer with n > 0, n < 0, a parent out of range).
 */
int cktlu_restart_closure(int32_t n, const int32_t *parent, const int32_t *unfinished, int32_t *in_set);

/*
 * The sets of this context's last pivot-check fallback (Section IV-C), host
 * out, int32[n] each, either may be NULL: unfinished[k] = 1 for the columns
 * the device had not finished when the check failed (every column of the
 * level whose check failed first and of later levels, and the dense-block
 * columns from the first failing one on), in_set the restart set computed
 * from them.  Which columns are unfinished depends only on the values, not on
 * the order in which the device ran its work.  Errors: E_ARG, E_STATE (no
 * fallback since the last cktlu_analyze).
 */
int cktlu_get_last_restart(const cktlu_ctx *ctx, int32_t *unfinished, int32_t *in_set);

/* Permutations (host out, int32[n] each): A(rowperm[k], colperm[j]) is the
 * (k, j) entry of the matrix that was factored, rowperm including pivoting. */
int cktlu_get_perm(const cktlu_ctx *ctx, int32_t *rowperm, int32_t *colperm);

/* Pre-processing result (host out, int32[n] each, any may be NULL): the
 * pre-processed matrix is A_hat(i, j) = A(rowperm_pre[i], colperm[j]); pivrow
 * is the pivot sequence (position k holds A_hat row pivrow[k]); parent is the
 * column elimination tree of A_hat (-1 = root). */
int cktlu_get_analysis(const cktlu_ctx *ctx, int32_t *rowperm_pre, int32_t *colperm,
                       int32_t *pivrow, int32_t *parent);

/* Sizes of the stored factors: strictly-lower L and U including diagonal. */
int cktlu_get_factor_nnz(const cktlu_ctx *ctx, int64_t *nnz_l, int64_t *nnz_u);

/* Factors of the last (re)factorization, host out, position-indexed CSC with
 * sorted rows: Lp[n+1], Li/Lx[nnz_l] (unit diagonal not stored), Up[n+1],
 * Ui/Ux[nnz_u] (diagonal last in each column).  Any pointer may be NULL.
 * instance selects a batched instance (0 otherwise).  Synchronises the stream. */
int cktlu_get_factors(cktlu_ctx *ctx, int32_t instance, int32_t *Lp, int32_t *Li, double *Lx,
                      int32_t *Up, int32_t *Ui, double *Ux);

/* Level of every column in the dependency graph of the current pattern
 * (Section II-B), host out int32[n]; sources are level 0. */
int cktlu_get_levels(const cktlu_ctx *ctx, int32_t *level);

/* Counters and sizes. */
int cktlu_get_stats(const cktlu_ctx *ctx, cktlu_stats *out);

/* Accumulated phase times (see cktlu_timing); synchronises the context's stream.
 * reset != 0 clears the accumulators afterwards.  Errors: E_ARG. */
int cktlu_get_timing(cktlu_ctx *ctx, cktlu_timing *out, int reset);

/* Device memory the context holds now, plus what one batched instance would
 * add (for admission control). */
size_t cktlu_footprint_bytes(const cktlu_ctx *ctx, int32_t batch);

/* ------------------------------------------------------------------------
 * Request loop (continuous serving of Newton-Raphson sequences).
 * A server owns `slots` worker threads, each with a HIP stream of default
 * priority.  Requests are taken in submission order; each is analysed and
 * factored on the host (cktlu_analyze, cktlu_factorize_host with its first
 * step's values), admitted once cktlu_footprint_bytes of it fits the HBM budget
 * next to the requests already resident (a request larger than the budget runs
 * alone), runs its steps (cktlu_refactorize + cktlu_solve per step) on its
 * slot's stream, so the work of different requests overlaps on the device, and
 * releases its memory.  A request computes exactly what a single context
 * would, whatever else is in the mix.  For callers that serve many circuits.
 * ---------------------------------------------------------------------- */
typedef struct cktlu_server cktlu_server;

typedef struct {
    int slots;                /* requests on the device at once (worker threads); default 4, 1..64 */
    double hbm_budget_bytes;  /* device bytes the resident requests may use together;
                                 0 (default) = 80% of the free HBM at creation */
    cktlu_options lu;         /* options of every request (precision, eps, ...); stream, timing and
                                 sweep_slot_map ignored (requests run without the slot map: their few
                                 steps do not repay building it) */
} cktlu_server_options;

typedef struct {
    int32_t n;                /* order of the circuit matrix */
    const int32_t *colptr;    /* host CSC pattern, colptr[n+1] and rowind[colptr[n]]; copied by submit */
    const int32_t *rowind;
    int32_t nsteps;           /* Newton-Raphson steps */
    const double *values_dev; /* device, nsteps x nnz: values of step t at t * nnz (caller-owned) */
    const double *b_dev;      /* device, n: right-hand side of every step */
    double *x_dev;            /* device, nsteps x n: solution of step t at t * n (written) */
    double arrival_s;         /* arrival time on the server clock (cktlu_server_now), for latencies */
    int64_t tag;              /* caller's identifier, returned with the completion */
} cktlu_request;

typedef struct {
    int64_t tag;
    int status;               /* 0, the first warning of its calls, or the first error (then it stopped) */
    double arrival_s;         /* server clock: arrival, taken by a slot, admitted to the device, finished */
    double start_s, admit_s, end_s;
    int32_t repivots;         /* steps whose pivot check failed (re-pivoted by the fallback) */
    int32_t fp64_fallbacks;   /* FP32_IR solves that fell back to FP64 */
    double backward_err;      /* FP32_IR: eta_inf of the last solve; -1 otherwise */
    size_t footprint;         /* device bytes it was admitted with */
} cktlu_request_done;

void cktlu_server_default_options(cktlu_server_options *opt);
/* Start the worker threads on the current HIP device.  Errors: E_ARG, E_NOMEM, E_HIP. */
int cktlu_server_create(cktlu_server **out, const cktlu_server_options *opt);
/* Queue a request (non-blocking).  Its device buffers must stay valid until its
 * completion is polled.  Errors: E_ARG, E_STATE (server stopping). */
int cktlu_server_submit(cktlu_server *srv, const cktlu_request *req);
/* Move up to max completions into out, waiting up to wait_ms for the first;
 * returns how many (>= 0) or E_ARG. */
int cktlu_server_poll(cktlu_server *srv, cktlu_request_done *out, int32_t max, int32_t wait_ms);
/* Seconds since the server was created (steady clock). */
double cktlu_server_now(const cktlu_server *srv);
/* Finish every queued request, stop the workers and release the server.  NULL is ignored. */
void cktlu_server_destroy(cktlu_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* CKTLU_H */
