/*
 * tacho.h -- C ABI of the MI355X (gfx950) supernodal multifrontal sparse
 * Cholesky library.
 *
 * The library solves A x = b for a sparse symmetric positive definite A in
 * the three phases of the paper's Trilinos section (symbolic analysis,
 * numerical setup, solve), with the Tacho section's method: a multifrontal
 * factorization P A P^T = L L^T scheduled by levels of the supernodal
 * elimination tree, followed by supernodal forward and backward
 * substitution scheduled by the same levels, with the diagonal blocks applied
 * through their explicit inverses (the inverted-diagonal-block solve variant
 * of that section).  Symbolic analysis runs on the host (it uses only the sparsity
 * pattern and is reused across value changes); the numeric phase and the
 * solves run in HIP kernels on the GPU.
 *
 * Conventions for every call:
 *   - Return value: TACHO_OK (0) or one of the negative TACHO_ERR_* codes;
 *     tacho_strerror() names them, tacho_last_error() gives a message for
 *     the calling thread's most recent failure.
 *   - Host pointers are read during the call only; the library copies what
 *     it keeps.  Device pointers must be valid on the given stream until the
 *     work queued by the call has finished.
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  All device
 *     work of a call is queued on it.
 *   - A handle serves one call at a time; different handles may be used
 *     concurrently from different threads on different streams.
 *   - Dense blocks (right-hand sides, solutions) are column-major with a
 *     leading dimension ld >= n.
 */
#ifndef TACHO_MI355X_H
#define TACHO_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TACHO_OK 0
#define TACHO_ERR_INVALID (-1) /* bad argument or malformed CSR */
#define TACHO_ERR_PATTERN (-2) /* pattern not structurally symmetric */
#define TACHO_ERR_NOT_SPD (-3) /* non-positive or NaN pivot */
#define TACHO_ERR_NOMEM (-4)   /* out of device memory or over the HBM budget */
#define TACHO_ERR_HIP (-5)     /* a HIP runtime call failed */
#define TACHO_ERR_SINGULAR (-6) /* LDL^T: a diagonal block has no usable pivot */

/* Precision of the numeric factorization (the paper's templated scalar
 * types, Trilinos section, and iterative refinement with computed factors,
 * Basker section). */
#define TACHO_FP64 0    /* FP64 fronts, FP64 solves */
#define TACHO_FP32_IR 1 /* FP32 fronts; tacho_solve refines in FP64 */
#define TACHO_FP32 TACHO_FP32_IR
/* Symmetric indefinite LDL^T in FP64 (Tacho section: besides Cholesky, an
 * LDL^T factorization of a symmetric indefinite matrix, with pivots searched
 * only within each diagonal block).  P A P^T = Q L D L^T Q^T: L unit lower
 * triangular with the supernodal structure of the Cholesky factor, D block
 * diagonal with 1x1 and 2x2 blocks, Q a permutation that moves a column only
 * within its diagonal block (the pivot columns of a supernode, cut into
 * blocks of at most 64 columns; 2x2 blocks never straddle two of them).
 * Pivots by Bunch-Kaufman partial pivoting, alpha = (1 + sqrt 17) / 8, with
 * the candidate rows and columns limited to the block's columns not yet
 * eliminated; ties go to the smallest index.  A block without a usable pivot
 * gives TACHO_ERR_SINGULAR.  Solves use the same sweeps as Cholesky with D^{-1}
 * applied between them; no refinement. */
#define TACHO_LDLT 2
/* LU of a general (nonsymmetric-valued) matrix with a symmetric pattern, FP64
 * (paper, Tacho section: LU is among the factorization types, pivots are
 * searched only within each diagonal block).  values hold every stored entry
 * of the caller's pattern (the analysis symmetrizes the pattern; entries it
 * adds are zero).  Q P A P^T = L U with L unit lower triangular, U upper
 * triangular and Q a row permutation that moves a row only within its
 * diagonal block (the same blocks as TACHO_LDLT: relaxed supernodes cut into
 * pieces of at most 64 columns); the pivot of column k is the entry of largest
 * magnitude among the block's rows k and below (ties to the first row); rows
 * below the block are never candidates.  A column whose candidates are all
 * zero gives TACHO_ERR_SINGULAR (fail_index: its original column).  Solves use
 * the Cholesky sweeps, forward on L and backward on U; no refinement, block
 * inverse solve variant only. */
#define TACHO_LU 3

/* Test hooks (tacho_options.debug_flags). */
#define TACHO_DEBUG_SOLVE_GIVE_UP 1 /* every solve raises its own hang flag before its
                                       launches, so each dependency wait gives up at once
                                       (the kernels still run to the end, the result is
                                       invalid); the error path is then reported like a
                                       real timed-out wait */

typedef struct tacho_sym *tacho_sym_t;
typedef struct tacho_num *tacho_num_t;

typedef struct {
  int32_t nd_leaf_size;      /* nested dissection stops at parts of at most this many
                                vertices (default 8) */
  int32_t small_front;       /* reserved, must be 0: fronts with m <= 64 are always
                                assembled and factored in LDS by one workgroup (the
                                class is fixed by the kernels' LDS layout) */
  int32_t scale_fp32;        /* FP32 path: symmetric Jacobi scaling diag(C)^{-1/2} (default 1) */
  int32_t refine_max;        /* FP32 path: at most this many corrections (default 10) */
  double refine_tol;         /* FP32 path: stop when ||b - A x||_2 / ||b||_2 <= tol
                                for every column (default 1e-10) */
  double stall_ratio;        /* FP32 path: a step with rho_k > stall_ratio * rho_{k-1},
                                twice in a row, counts as a stall (default 0.5) */
  uint64_t hbm_budget_bytes; /* 0 = no limit; tacho_factorize returns TACHO_ERR_NOMEM
                                when the factor plus workspace would exceed it */
  int32_t block_size;        /* reserved, must be 0: the pivot-block width of the
                                large-front kernels is 64 (their MFMA tiling) */
  int32_t ordering;          /* 0 (default): both orderings below, keep the one with
                                fewer factorization flops; 1: multilevel nested
                                dissection; 2: level-structure nested dissection */
  int32_t graphs;            /* 1 (default): the factorization's launch sequence is
                                captured once per numeric handle into a hipGraph and
                                replayed; 0: launched eagerly.  Kernel profiling
                                always launches eagerly. */
  int32_t front_kernel;      /* large fronts (m > 64): 0 (default) one dataflow launch
                                per level (tile tasks over 64-column pivot blocks with
                                completion counters); 1: stepwise launches per pivot
                                block (diagonal block, rows below, trailing update) */
  /* Batching parameters of the launch plan (0 = default, or the tuned value
   * when autotune_path is set).  They change how work is grouped into tasks
   * and launches, not which operations a front performs.  solve_level_fronts,
   * asm_cols and solo_m give bitwise the same results for every setting;
   * u_range, chain_min and chain_inplace change the order in which a front's
   * contributions are summed, so results agree to rounding.  The autotuner
   * of the Python package times candidates on the device. */
  int32_t u_range;           /* pivot blocks per update-matrix range task (default 8);
                                the dataflow plan forms update matrices in a launch of
                                their own after the panels, over all pivot blocks at
                                once, so it takes no ranges and this has no effect there */
  int32_t chain_min;         /* fronts with at least this many 64-column pivot blocks
                                run their diagonal blocks as one chain task (default 3;
                                negative: never) */
  int32_t solve_level_fronts; /* solve levels below the last level with more than
                                this many fronts run level by level (default 256) */
  int32_t asm_cols;          /* front columns per assembly work item of a front taller
                                than 4096 rows (default 8; shorter fronts get whole
                                columns, as many as fit in 4096 entries, at most 64) */
  int32_t solo_m;            /* fronts with one pivot block (w <= 64) and at most this
                                many rows run as one task each, without completion
                                flags (default 192; negative: never) */
  int32_t chain_inplace;     /* chain fronts: the product for the next diagonal block's
                                row tile is subtracted in place by the tasks that form
                                it (>= 0, default) or left in a slot for the chain (< 0) */
  int32_t debug_flags;       /* TACHO_DEBUG_* test hooks (default 0) */
  const char *autotune_path; /* NULL (default) or the path of the autotuner's JSON table,
                                read by tacho_analyze: batching parameters left at 0 take
                                the table's values, the order-neutral ones (asm_cols,
                                solo_m, solve_level_fronts) from the entry of the
                                workload class "n~2^<lg>/deg<d>/<fp64|fp32>" (lg the
                                integer nearest log2(n), d = nnz/n rounded), the
                                order-changing ones (u_range, chain_min, chain_inplace)
                                from the entry "order/<fp64|fp32>", which does not depend
                                on the workload, so that a system factored alone and in a
                                batch gets the same arithmetic.  Absent entries leave the
                                defaults; an unreadable or malformed file is
                                TACHO_ERR_INVALID.  The string is read during the call. */
  int32_t autotune_precision; /* which precision's table entries to take (TACHO_FP64,
                                default, or TACHO_FP32): a symbolic handle holds one
                                launch plan, used by numeric handles of either precision */
  /* Condensed graph of the symbolic analysis (Tacho section: analysis on a
   * graph compressed by the DOFs of each grid point).  The ordering runs on the
   * condensed graph and keeps each condensed vertex's rows consecutive, so
   * they share a supernode; when every condensed vertex's rows are
   * indistinguishable (equal pattern rows), the elimination tree and column
   * counts are derived from the condensed graph's (weighted by the number of
   * rows), otherwise they are computed on the full pattern.  Either way the
   * symbolic result is that of P A P^T with the resulting P. */
  int32_t dof_block;         /* 0 (default): condense indistinguishable rows found in the
                                pattern; 1: no condensation; b >= 2: rows [k b, (k+1) b)
                                form condensed vertex k (b must divide n) */
  const int32_t *dof_map;    /* NULL (default) or n entries: the condensed vertex of each
                                row, ids 0..nc-1 all used; overrides dof_block; not
                                accepted by tacho_analyze_batch.  Read during the call. */
} tacho_options;

/* Fill `opt` with the defaults listed above. */
void tacho_default_options(tacho_options *opt);

typedef struct {
  int64_t n;                /* order of A */
  int64_t nnz_a;            /* stored entries of the full symmetric pattern (plus added
                               diagonal entries) */
  int64_t nnz_l;            /* sum_j eta_j: entries of L including the diagonal */
  int64_t flops;            /* sum_j eta_j^2: algorithmic factorization flops */
  int64_t nsuper;           /* relaxed supernodes */
  int64_t nlevels;          /* height of the supernodal elimination forest + 1 */
  int64_t max_front;        /* largest front order m */
  int64_t max_width;        /* largest supernode width w */
  int64_t factor_bytes_fp64; /* device bytes of the FP64 factor panels */
  int64_t work_bytes_fp64;  /* peak device bytes of the FP64 update matrices */
  int64_t device_bytes_fp64; /* all device memory of one FP64 numeric handle (nrhs = 1) */
  int64_t nsystems;         /* independent systems (1 unless built by tacho_analyze_batch) */
  int64_t nnz_factor;       /* stored factor entries: nnz_l plus the explicit zeros of
                               relaxed supernodes */
  int64_t ordering;         /* ordering used: 1 multilevel, 2 level-structure; a batch
                               orders each system alone (3: its systems used both) */
  int64_t t_order_us;       /* host microseconds of the analysis: fill-reducing ordering */
  int64_t t_structure_us;   /* etree, counts, supernodes, row structures, maps, levels */
  int64_t t_plan_us;        /* launch plan, memory plan and refinement maps */
  /* batching parameters of the launch plan in effect (defaults and table resolved;
     plan_chain_inplace 1 = in place, -1 = slot) */
  int64_t plan_u_range, plan_chain_min, plan_solve_level_fronts, plan_asm_cols, plan_solo_m,
      plan_chain_inplace;
} tacho_sym_info;

typedef struct {
  int32_t iters;      /* FP32 path: refinement corrections applied (0 for FP64) */
  int32_t fell_back;  /* FP32 path: 1 if the FP32 factorization broke down or
                         refinement stalled, and the solve was done with an FP64
                         refactorization of the same values (still a success) */
  double relres_max;  /* max over columns of ||b - A x||_2 / ||b||_2 (FP32 path) */
  double *relres;     /* optional, caller-owned array of nrhs entries receiving the
                         per-column relative residual (FP32 path), or NULL */
  int32_t *fell_back_units; /* optional, caller-owned array of nsystems * nrhs entries
                         (system index fastest) receiving 1 where that system's
                         column took the FP64 factor's solution, else 0 (FP32 path) */
} tacho_solve_info;

/*
 * Symbolic analysis (Trilinos section, step 1: pattern only, done once per
 * pattern on one host core; Tacho section: nested-dissection reordering, as
 * the land-ice runs use METIS).
 *   n        order of A (n >= 0)
 *   rowptr   host int64[n+1], 0-based CSR row pointers, rowptr[0] = 0
 *   colind   host int32[rowptr[n]], column indices of the FULL symmetric
 *            pattern; unsorted rows are accepted, duplicates are rejected
 *            (TACHO_ERR_INVALID), a structurally unsymmetric pattern gives
 *            TACHO_ERR_PATTERN; a missing diagonal entry is added
 *   opt      options or NULL for the defaults
 *   out      receives the symbolic handle (owned by the caller, released with
 *            tacho_free_symbolic)
 * The handle holds: the fill-reducing permutation (own nested dissection,
 * composed with an elimination-tree postorder), the elimination tree, the
 * column counts, relaxed supernodes (fundamental supernodes merged up a
 * chain while the explicit zeros of the merged dense block stay under a
 * size-dependent fraction: 1/2 for fronts of order <= 16, 1/5 up to 64,
 * 1/20 above), their row structures, the
 * child-to-parent relative maps, the A-entry-to-front maps, the level
 * schedule and the device memory plan.  No device work is queued.
 */
int tacho_analyze(int64_t n, const int64_t *rowptr, const int32_t *colind,
                  const tacho_options *opt, tacho_sym_t *out);

/*
 * Symbolic analysis of `nsys` independent systems solved together (the
 * single-GPU analogue of the many MPI ranks per GPU of the paper's land-ice
 * runs).  System k has order n[k] and CSR arrays rowptr[k], colind[k] as in
 * tacho_analyze.  The handle represents the block-diagonal matrix of all
 * systems in order; values, right-hand sides and solutions are the
 * concatenation of the systems' arrays.  Each level of the merged
 * elimination forest is factored by one launch sequence for all systems.
 */
int tacho_analyze_batch(int64_t nsys, const int64_t *n, const int64_t *const *rowptr,
                        const int32_t *const *colind, const tacho_options *opt,
                        tacho_sym_t *out);

/* Scalars of a symbolic handle. */
int tacho_query_symbolic(tacho_sym_t sym, tacho_sym_info *info);

/*
 * Copies of the symbolic arrays (any pointer may be NULL):
 *   perm[n]          new -> old: row/column i of P A P^T is row/column perm[i] of A
 *   parent[n]        elimination tree of P A P^T, -1 for roots
 *   colcount[n]      eta_j, nonzeros of column j of L including the diagonal
 *   super_ptr[ns+1]  first column of each (relaxed) supernode the factor is stored in
 *   super_parent[ns] supernodal parent, -1 for roots
 *   level[ns]        level (height) of each supernode, leaves are 0
 */
int tacho_get_symbolic(tacho_sym_t sym, int32_t *perm, int32_t *parent, int64_t *colcount,
                       int32_t *super_ptr, int32_t *super_parent, int32_t *level);

/*
 * Numerical factorization (Trilinos section, step 2; Tacho section:
 * multifrontal Cholesky with level-set scheduling).
 *   sym               symbolic handle (must outlive the numeric handle)
 *   values            float64[nnz] aligned with the colind given to
 *                     tacho_analyze (concatenated per system for a batch);
 *                     only entries with row >= column are read, numerical
 *                     symmetry is the caller's contract
 *   values_on_device  0: host pointer; 1: device pointer used on hip_stream
 *   precision         TACHO_FP64, TACHO_FP32, TACHO_LDLT or TACHO_LU
 *   out               receives the numeric handle, which owns the device factor
 *   fail_index        optional; on TACHO_ERR_NOT_SPD receives the original
 *                     index of the first column (in elimination order) whose
 *                     pivot was not positive; no handle is created then
 * Blocks the calling thread until the device work is finished (one
 * device-to-host read of the failure flag).  With TACHO_FP32 a pivot
 * breakdown of the FP32 factorization is not an error: the same values are
 * refactored in FP64 on the same symbolic handle and the solves use that
 * factor (info->fell_back = 1); TACHO_ERR_NOT_SPD is returned only when the
 * FP64 factorization fails too.
 */
int tacho_factorize(tacho_sym_t sym, const double *values, int values_on_device, int precision,
                    void *hip_stream, tacho_num_t *out, int64_t *fail_index);

/*
 * Allocate a numeric handle without factoring (for callers that queue the
 * factorization asynchronously with tacho_refactorize(..., sync = 0), such as
 * a request server).  The handle holds no factor until then; solving before
 * gives TACHO_ERR_INVALID.
 */
int tacho_numeric_create(tacho_sym_t sym, int precision, tacho_num_t *out);

/* Device bytes a numeric handle of this precision allocates (factor, update
 * workspace, values, solve workspace for 16 right-hand sides); the quantity an
 * HBM budget is checked against. */
int tacho_numeric_bytes(tacho_sym_t sym, int precision, int64_t *bytes);

/*
 * Refactorization with new values on the same pattern (Trilinos section:
 * the symbolic analysis is amortized across value changes).  Same arguments
 * as tacho_factorize; the handle keeps its precision and device memory.  On
 * TACHO_ERR_NOT_SPD the handle stays valid but holds no usable factor.
 * With `sync` = 0 the call returns without waiting and the failure flag is
 * read by the next tacho_solve or tacho_check_factor.
 */
int tacho_refactorize(tacho_num_t num, const double *values, int values_on_device,
                      void *hip_stream, int sync, int64_t *fail_index);

/*
 * Wait for the last factorization of `num` and report its failure flag, then
 * wait for the last solve queued on the handle (on the stream it was queued
 * on) and report TACHO_ERR_HIP if one of its dependency waits timed out (its
 * result is then invalid).  A reported timeout is cleared, so the handle's
 * next solve runs normally.
 */
int tacho_check_factor(tacho_num_t num, int64_t *fail_index);

/*
 * Solve A X = B (Trilinos section, step 3; Tacho section, supernodal
 * triangular solves: level-set scheduled forward and backward substitution
 * over the dense supernodal blocks, each 64-column diagonal block applied
 * through its explicit inverse, which the factorization keeps; several
 * right-hand sides at once use block operations).
 *   b, x        n x nrhs column-major blocks with leading dimension ld >= n;
 *               x may equal b (in place)
 *   on_device   0: host pointers; 1: device pointers used on hip_stream
 *   info        optional refinement report (see tacho_solve_info)
 * For an FP32 factor the solve refines in FP64: x = solve32(b), then
 * r = b - A x (FP64 sparse product), x += solve32(r) until the relative
 * residual of every column is <= refine_tol.  Convergence is tracked per
 * system and column; a column that stalls (or belongs to a system whose FP32
 * factorization broke down) is refactored in FP64 on the same symbolic handle
 * and takes the FP64 solution, while the other columns keep their refined
 * results (info->fell_back, info->fell_back_units).
 * Blocks until the result is available when on_device = 0 or for the FP32
 * path; the FP64 device path only queues work, also behind a factorization
 * queued with sync = 0 (whose failure flag tacho_check_factor then reports).
 */
int tacho_solve(tacho_num_t num, const double *b, double *x, int64_t nrhs, int64_t ld,
                int on_device, void *hip_stream, tacho_solve_info *info);

/*
 * tacho_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, queued on hip_stream, that calls no hipMalloc/hipFree.
 *   b, x   DEVICE pointers, n x nrhs column-major with leading dimension
 *          ld >= n.  With an FP64 factor x may equal b.  With an FP32 factor
 *          (refinement) ld must equal n, x must differ from b, nrhs <= 16,
 *          and the refinement's scratch (8 n nrhs bytes of residual, as many
 *          again for the iterate by rows when nrhs > 1, 1041 nsystems nrhs
 *          bytes of norms, their partial sums and a mask) must fit the
 *          library's fixed device array of 64 MiB per GPU; otherwise
 *          TACHO_ERR_INVALID.
 * The scratch array is shared by every call on a GPU and keeps the last
 * call's contents: calls that overlap on one GPU (different streams or
 * threads) race and must be serialized by the caller.  If refinement would
 * need the FP64 fallback factor and the handle does not hold one yet (an
 * FP32 breakdown or stall), the call returns TACHO_ERR_NOMEM instead of
 * allocating it; tacho_solve then does the fallback.  Blocking behaviour and
 * `info` are those of tacho_solve with on_device = 1.
 */
int tacho_solve_noalloc(tacho_num_t num, const double *b, double *x, int64_t nrhs, int64_t ld,
                        void *hip_stream, tacho_solve_info *info);

/*
 * Solve variant (Tacho section, the SpTRSV variants).  Both apply inverses of
 * diagonal blocks:
 *   TACHO_SOLVE_BLOCK_INVERSE (default): each supernode's diagonal part in
 *     64-column blocks with their stored inverses (the inverted-diagonal-block
 *     variant); the blocks of one supernode follow each other.
 *   TACHO_SOLVE_PARTITIONED_INVERSE: the partitioned inverse, L^-1 as the
 *     product over the levels of the inverses of L's level-l part; every
 *     supernode's panel [L11; L21] becomes [L11^-1; L21 L11^-1], and a sweep
 *     is one merged matrix-vector product per supernode, one gather and one
 *     product launch per level.  Its setup costs about the factorization's
 *     off-diagonal work (sum over supernodes of m w^2 flops) and as much
 *     device memory again as the factor L (plus 128 n bytes and the sweeps'
 *     partial products of long supernodes); its accuracy
 *     depends on the condition of each supernode's L11.
 *   TACHO_SOLVE_LEVEL_CSR: the same partitioned inverse stored as one
 *     compressed-sparse-row matrix per level and sweep (rows of the solve
 *     vector, 32-bit column indices), one sparse matrix-vector product per
 *     level and sweep on the whole solve vector (no gathers, no update
 *     vectors; an ancestor row adds the terms of all the level's fronts that
 *     hold it, in front order).  Its setup is the partitioned inverse's plus
 *     a copy; it keeps the inverse panels and adds about twice nnz(L) entries
 *     of (value, index) (rows of both sweeps).
 * tacho_set_solve_variant selects the variant of later tacho_solve calls on
 * `num`.  Choosing TACHO_SOLVE_PARTITIONED_INVERSE or TACHO_SOLVE_LEVEL_CSR
 * waits for the handle's factorization, builds the inverse panels (and the
 * CSR copy) on hip_stream and waits for them; every later factorization of
 * the handle (tacho_refactorize) rebuilds them on its stream.  The CSR
 * form needs 2 n < 2^31.  Cholesky handles (TACHO_FP64, TACHO_FP32) only: TACHO_LDLT
 * returns TACHO_ERR_INVALID, as does an unknown variant; TACHO_ERR_NOMEM if
 * the extra memory exceeds options.hbm_budget_bytes.  An FP32 handle's
 * refinement solves use it too; its FP64 fallback factor keeps the default.
 */
#define TACHO_SOLVE_BLOCK_INVERSE 2
#define TACHO_SOLVE_PARTITIONED_INVERSE 3
#define TACHO_SOLVE_LEVEL_CSR 4
int tacho_set_solve_variant(tacho_num_t num, int variant, void *hip_stream);

/*
 * Copy the factor L (of P A P^T, FP64 or FP32 widened to FP64) to host CSC
 * arrays as stored: Lp int64[n+1], Li int32[nnz_factor], Lx
 * float64[nnz_factor]; every column sorted ascending with the diagonal
 * first; rows that are structurally zero in L but stored in a relaxed
 * supernode hold exact zeros.  Synchronizes the handle.  After an FP32 pivot
 * breakdown the FP32 factor is not valid and the FP64 factor of the same
 * values (the one the solves fall back to) is returned.
 */
int tacho_get_factor(tacho_num_t num, int64_t *Lp, int32_t *Li, double *Lx);

/*
 * D and the pivot order of a TACHO_LDLT factorization (any pointer may be
 * NULL; host arrays of n entries, permuted numbering of P A P^T):
 *   d[k]  diagonal of D
 *   e[k]  subdiagonal of D: nonzero exactly at the first column k of a 2x2
 *         pivot block (coupling k and k + 1), zero elsewhere
 *   q[i]  row i of L is row q[i] of P A P^T (q permutes within diagonal blocks)
 * L itself comes from tacho_get_factor (unit diagonal stored explicitly; the
 * entry below the first column of a 2x2 pivot is zero).  Synchronizes.
 */
int tacho_get_ldlt(tacho_num_t num, double *d, double *e, int32_t *q);

/*
 * U and the row order of a TACHO_LU factorization (host arrays, permuted
 * numbering of P A P^T):
 *   Up, Ui, Ux  U^T in the layout of tacho_get_factor (Up: n + 1 column
 *               pointers, column c lists U's row c: column indices j >= c of U
 *               in ascending order, the diagonal first; all three NULL, or all
 *               three sized like tacho_get_factor's)
 *   q[i]        row i of L U is row q[i] of P A P^T (NULL: not returned)
 * L comes from tacho_get_factor (unit diagonal stored explicitly, rows in the
 * order of L U).  Synchronizes.  TACHO_ERR_INVALID for other precisions.
 */
int tacho_get_lu(tacho_num_t num, int64_t *Up, int32_t *Ui, double *Ux, int32_t *q);

/* Device milliseconds of the last factorization and solve (hipEvent timing on the
 * caller's stream; valid once that work has finished). */
int tacho_last_times(tacho_num_t num, double *factor_ms, double *solve_ms);

/*
 * Kernel profiling.  While enabled, every kernel launch of the handle's
 * factorizations and solves is bracketed by hipEvents on the caller's stream
 * (adding a little launch overhead), and its algorithmic flops and bytes are
 * taken from the launch plan: dense partial factorization sum_{j<w}(m-j)^2
 * per front, lower-triangle updates 2*K*(outputs with row >= col), solves
 * 2 flops per factor entry and right-hand side, bytes counting each factor
 * entry, A entry and update-matrix entry once.  Kinds:
 */
#define TACHO_K_SMALL_FRONT 0 /* fronts assembled and factored in LDS */
#define TACHO_K_ASSEMBLE 1    /* large-front assembly and extend-add */
#define TACHO_K_DIAG 2        /* diagonal-block Cholesky of a panel */
#define TACHO_K_PANEL 3       /* triangular solve of the rows below a panel */
#define TACHO_K_UPDATE 4      /* matrix-core lower-triangular updates (SYRK/GEMM) */
#define TACHO_K_GATHER 5      /* A values into assembly order */
#define TACHO_K_FORWARD 6     /* forward substitution, one launch per level */
#define TACHO_K_BACKWARD 7    /* backward substitution, one launch per level */
#define TACHO_K_PERMUTE 8     /* right-hand side / solution permutation */
#define TACHO_K_REFINE 9      /* FP64 residual and norms of the refinement */
#define TACHO_K_FRONT 10      /* dataflow factorization of a level's large fronts */
#define TACHO_K_PINV 11       /* partitioned-inverse setup (tacho_set_solve_variant) */
#define TACHO_PROFILE_KINDS 12

/* enable = 1 clears the counters and starts recording; 0 stops. */
int tacho_profile(tacho_num_t num, int enable);
/* Totals for one kind since profiling was enabled (waits for the events). */
int tacho_profile_read(tacho_num_t num, int kind, int64_t *launches, double *ms, double *flops,
                       double *bytes);
/* Name of the HIP kernel behind a profiling kind. */
const char *tacho_kernel_name(int kind);

int tacho_free_symbolic(tacho_sym_t sym);
int tacho_free_numeric(tacho_num_t num);
const char *tacho_strerror(int code);
const char *tacho_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TACHO_MI355X_H */
