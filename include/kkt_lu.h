/*
 * kkt_lu.h - fixed-pattern sparse LU refactorization and solve for sequences
 * of same-pattern KKT systems, FP64, on one AMD MI355X (gfx950).
 *
 * The operations follow the paper's problem statement and solver phases:
 *   - a sequence K_k x_k = r_k whose matrices all share one sparsity pattern
 *     (Section 2, eq. "eq:kktlinear" and the paragraph after it);
 *   - three phases, symbolic / numeric / solve, with the pivot sequence and
 *     factor patterns of the first system reused for all later ones
 *     (Section 4, the "refactorization" discussion);
 *   - the first system analysed on the CPU and everything after it on the
 *     GPU, data moved to the device once (Section 5 introduction and 5.1.2);
 *   - refinement as flexible GMRES with re-orthogonalized classical
 *     Gram-Schmidt, LU factors as the preconditioner, workspaces allocated
 *     once (Section 5.1.1 and 5.1.2).
 *
 * Conventions shared by every entry point:
 *   Matrices are square CSR, 0-based, int64 row pointers, int32 column
 *   indices, columns sorted ascending within a row, no duplicates.  Both
 *   triangles of a symmetric KKT matrix are stored; the library treats it as
 *   a general matrix.
 *   Q[k] is the original index of the k-th eliminated vertex, A' = Q^T A Q
 *   (A'[k][l] = A[Q[k]][Q[l]]); P[k] is the A'-row chosen as pivot at step k;
 *   P A' = L U with L unit lower triangular, U upper triangular.
 *   Dense vectors with several right-hand sides are column-major n x nrhs.
 *   Pointers named d_* are device pointers (hipMalloc'ed or torch CUDA
 *   tensors); all others are host pointers.  `stream` is a hipStream_t
 *   (NULL = the legacy default stream).
 *
 * Ownership: the caller owns every buffer it passes.  kkt_analyze copies what
 * it needs from host arrays.  The handle owns all device workspaces; they are
 * allocated by kkt_analyze and reused by every later call.  Device pointers
 * passed to kkt_refactor / kkt_solve / kkt_grad_values are read or written in
 * stream order and must stay valid until that work completes.
 *
 * Errors: negative status = fatal, nothing was changed; positive = warning,
 * the computation went on (the paper lets the first factorization continue on
 * a singular matrix, Section 5.1.2); kkt_last_error() gives a message.  No
 * C++ exception crosses this interface.  One host thread per handle at a
 * time.
 */
#ifndef KKT_LU_H
#define KKT_LU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kkt_ctx *kkt_handle;

typedef enum {
  KKT_OK = 0,
  KKT_WARN_NUMERICALLY_SINGULAR = 1, /* a pivot column was all zeros (analyze) */
  KKT_WARN_TINY_PIVOT = 2,           /* |u_kk| < tiny_pivot_rel * ||A||_inf or non-finite */
  KKT_WARN_NOT_CONVERGED = 3,        /* refinement budget spent before eta_target */
  KKT_WARN_PERTURBED_PIVOT = 4,      /* a pivot was raised to the static-pivoting threshold */
  KKT_WARN_REANALYZED = 5,           /* a solve re-ran the pivoting pass (auto_reanalyze) */
  KKT_ERR_INVALID_ARG = -1,
  KKT_ERR_BAD_PATTERN = -2,          /* unsorted / duplicate / out-of-range CSR */
  KKT_ERR_STRUCTURALLY_SINGULAR = -3,
  KKT_ERR_STATE = -4,                /* e.g. refactor before analyze */
  KKT_ERR_OUT_OF_MEMORY = -5,
  KKT_ERR_DEVICE = -6,               /* a HIP runtime call failed */
  KKT_ERR_NONFINITE = -7,            /* NaN/Inf in analyze's values; from kkt_sync_report: in
                                        the last refactorization's values (their NaNs enter
                                        the factors as quiet NaNs) */
  KKT_ERR_TOO_LARGE = -8             /* factor size exceeds the int32 index range */
} kkt_status;

typedef struct {
  int32_t ordering;         /* 0 exact minimum degree on A+A^T (default), 1 natural, 2 user Q */
  double pivot_tau;         /* threshold partial pivoting in (0,1]; 1e-10 = KKT preset (default) */
  int32_t fgmres_restart;   /* Krylov restart length, default 20 */
  int32_t fgmres_max_iters; /* total refinement iterations per right-hand side, default 20 */
  int32_t min_iters;        /* always run at least this many iterations, default 0 */
  double eta_target;        /* stop when ||b-Ax||_inf/(||A||_inf ||x||_inf) <= target, 1e-12 */
  double tiny_pivot_rel;    /* tiny-pivot warning threshold relative to ||A||_inf, 1e-18 */
  int32_t device;           /* HIP device ordinal, default 0 */
  int32_t schedule;         /* 0 auto, 1 level-synchronous launches, 2 dependency-driven */
  int32_t sync_mode;        /* dependency-driven publication: 0 default, 1 device-scope
                               acquire/release fences, 2 device-coherent accesses (the solution
                               value is its own ready flag in the triangular solves) */
  int32_t solve_entries_per_lane; /* triangular-solve chunking: lanes per row sized so each lane
                                     holds at most this many entries (0 = 8; 1..64) */
  int32_t refactor_waves_per_block; /* dependency-driven refactorization: 0 auto, 1, 2 or 4 */
  int32_t solve_thin_rows; /* single right-hand-side solves with device-coherent publication:
                              runs of levels with at most this many rows at either end of a
                              triangular schedule are solved by one workgroup with barriers
                              instead of cross-CU flags (0 = 16, -1 = never; at most 256) */
  int32_t dense_tail; /* dependency-driven refactorization: the trailing block of this many
                         pivots is finished as a dense LU (bitwise the same factors) and the
                         solves treat it as a dense triangle; 0 = auto (the largest block of
                         at least 256 and at most 2048 pivots that is at least half dense,
                         else none), -1 = never, at most 2048 */
  int32_t solve_blocks_per_cu; /* dependency-driven triangular solves: 256-thread workgroups
                                  per CU in the persistent grid (0 = 8; 1..8): fewer waves
                                  waiting ahead of the dependency front poll less */
  int32_t solve_chain; /* single right-hand-side solves with device-coherent publication:
                          longest run of chained rows (each depending on the one before)
                          solved by one wave (0 = 32, 1..32; -1 = no chain blocks: level
                          chunks plus one-workgroup thin segments) */
  int32_t refactor_map; /* dependency-driven refactorization: 0 = precomputed update positions
                           (one 16-bit entry per multiply-add of the factorization, built once
                           at analysis), -1 = binary search of each update's column instead */
  int32_t refactor_crit_height; /* dependency-driven refactorization: rows with at least this many
                                   rows chained after them are handed out first in their band
                                   (0 = 32, -1 = plain level order) */
  int32_t refactor_waves_per_cu; /* dependency-driven refactorization: cap on the resident waves
                                    per CU of its persistent grid (0 = occupancy limit) */
  int32_t refine; /* refinement method: 0 FGMRES-CGS2 (default), 1 classical iterative
                     refinement x <- x + M^{-1}(b - A x); both use fgmres_max_iters as the
                     iteration budget, min_iters and eta_target */
  int32_t auto_reanalyze; /* 1: a single-system solve that misses eta_target re-runs the pivoting
                             pass on the current matrix (kkt_reanalyze) and solves again once
                             (warning KKT_WARN_REANALYZED); 0 = off (default) */
  int32_t solve_jacobi_sweeps; /* > 0: op 'N' solves replace the exact triangular solves by
                                  this many Jacobi sweeps per triangle (approximate triangular
                                  solves; FGMRES absorbs the difference), 0 = exact (default) */
  int32_t refactor_short_rows; /* dependency-driven refactorization with device-coherent
                                  publication: 0 = rows of the short-row band (at most 256
                                  entries) take all their updates as one list loaded a window
                                  at a time (default), -1 = pivot by pivot like the other bands */
  double pivot_perturb_rel; /* static pivoting in the refactorizations: a pivot with
                               |u_kk| < pivot_perturb_rel * ||A||_inf becomes
                               copysign(pivot_perturb_rel * ||A||_inf, u_kk) (warning
                               KKT_WARN_PERTURBED_PIVOT; refinement corrects the solve);
                               0 = off (default), < 1 */
  int32_t refactor_long_rows; /* dependency-driven refactorization with device-coherent
                                 publication and update maps, rows outside the short-row band:
                                 0 = the pivot rows of the next steps are loaded into registers
                                 ahead of their steps and only the row's values are staged in LDS
                                 (default), -1 = each step loads its pivot row when it starts */
  int32_t refine_sync; /* 0 (default): the refinement's stop test runs on the device; kkt_solve
                         launches the direct solve, the test and a fixed budget of refinement
                         iterations (refine_budget) whose kernels return at once after the test
                         stopped them, and never waits for the device (graph-capturable);
                         1: the host reads eta back after every step and launches only the
                         iterations needed (kkt_solve then synchronises the stream) */
  int32_t refine_budget; /* refinement iterations launched per right-hand side when
                            refine_sync = 0: 0 = fgmres_max_iters (default), k > 0 =
                            min(k, fgmres_max_iters) (at least min_iters), -1 = adaptive:
                            2 r + 2 where r is the iteration count of the last earlier solve
                            whose outcome has reached the host without waiting, the full
                            budget after a solve that missed eta_target, after
                            kkt_update_matrix, and with static pivoting, Jacobi sweeps or
                            min_iters > 0 (graph captures always take the full budget).  A
                            solve that has not met eta_target within its budget reports
                            KKT_WARN_NOT_CONVERGED */
  int32_t dense_lu; /* dense trailing block's factorization: 0 = a panel launch and an update
                       launch per 32 pivots (default), 1 = one dependency-driven launch over
                       32 x 32 tiles with a look-ahead of one panel, then a copy of the factored
                       diagonal tiles; the same values */
  int32_t debug_spin_limit; /* testing: > 0 makes a dependency wait give up once the wave has
                               polled this many times (checked on its second poll and every 64th),
                               raising the stall flag, so every kernel drains and kkt_sync_report
                               returns KKT_ERR_DEVICE; 0 = off */
  int32_t debug_schedule;   /* testing: 1 = adversarial ticket schedule in the persistent kernels
                               (other workgroups take each chunk, pseudo-random pauses); results
                               are unchanged.  Process-wide on the device, set by the last
                               analysis; 0 = off */
  int32_t matching;         /* 1: before the ordering, a maximum-product matching of the nonzero
                               entries permutes the rows and power-of-two row and column
                               scalings from its dual potentials make the matched entries about 1
                               and every entry at most 2 in magnitude (Section 5.2.1's MC64-style
                               preprocessing); the factors are those of Ahat = Pm Dr A Dc, the
                               solves and residuals stay those of A.  Fixed at analysis (a
                               re-analysis keeps it); single systems only.  0 = off (default) */
  int32_t refactor_micro_rows; /* short-row band of the dependency-driven refactorization: 0 =
                                  rows of at most 8 entries, 4 pivots and 4 multiply-adds go
                                  one per lane, up to 64 rows of one level to a wave (default);
                                  -1 = one wave per row for every row of the band */
  int32_t debug_timeline;   /* profiling: 1 = every refactorization records, per row of its two
                               band kernels, when the row started, when it last found an input
                               missing and when its stores completed (kkt_debug_timeline);
                               0 = off (default) */
  int32_t refactor_short_band; /* dependency-driven refactorization: longest row of the short-row
                                  band (rows fed only by such rows go to the list kernel);
                                  0 = 128 (default), at most 256 */
} kkt_options;

typedef struct {
  int32_t warnings;  /* bit (1 << KKT_WARN_*) for every warning raised since the last report */
  int32_t iters;     /* refinement iterations of the last solve (max over right-hand sides) */
  double eta;        /* final eta of the last solve (max over right-hand sides) */
  double eta0;       /* eta right after the direct solve (max over right-hand sides) */
  double min_pivot;  /* min |u_kk| of the last refactorization */
  double max_pivot;  /* max |u_kk| of the last refactorization */
  double anorm_inf;  /* ||A||_inf of the last refactorization */
  double growth;     /* max |u_ij| over U / ||A||_inf of the last refactorization (pivot
                        growth; Section 5.1.1 re-analyses when the factors degrade) */
} kkt_report;

typedef struct {
  int32_t n;
  int64_t nnz;         /* nnz(A) */
  int64_t nnz_l;       /* strict lower part of the factors */
  int64_t nnz_u;       /* upper part including the diagonal */
  int32_t levels;      /* depth of the row dependency graph (refactor, L solve) */
  int32_t levels_u;    /* depth of the U-solve dependency graph */
  int32_t analyze_status; /* KKT_OK or KKT_WARN_NUMERICALLY_SINGULAR */
  int64_t device_bytes;   /* device memory owned by the handle */
  double analyze_seconds;
  int32_t dense_tail;     /* pivots in the dense trailing block (0 = none) */
  int64_t factor_epoch;   /* incremented by every call that replaces the factors or the
                             matrix (analyze, refactor, reanalyze, update_matrix, graph
                             launch); lets a caller tell whether saved solutions still
                             belong to the current factors */
  int32_t levels_sparse;  /* dependency levels of the rows outside the dense block (the
                             refactorization's row-to-row waits) */
  int32_t solve_block_levels[2]; /* dependency levels of the chain-blocked L and U solves
                             over the rows outside the dense block: a run of chained rows
                             solved by one wave counts once; 0 where that path is off */
} kkt_info;

/* Fill *opt with the defaults listed above. */
void kkt_options_default(kkt_options *opt);

/* Create a handle bound to opt->device (opt may be NULL for defaults).
 * Returns KKT_ERR_INVALID_ARG for out-of-range options. */
kkt_status kkt_create(const kkt_options *opt, kkt_handle *out);
kkt_status kkt_destroy(kkt_handle h);

/* Symbolic + pivoting analysis of the first matrix on the host, then one
 * upload of every index structure to the device (Sections 4 and 5.1.2).
 * Orders pattern(A+A^T) (opt->ordering), runs a left-looking LU with
 * threshold partial pivoting on A' using values0 to fix P, derives the L/U
 * patterns, the A->LU value map and the dependency schedules.  user_q (n
 * entries) is read only when opt->ordering == 2.  Synchronous.  Re-analysing
 * a handle replaces its previous analysis.
 * Errors: INVALID_ARG, BAD_PATTERN, NONFINITE, STRUCTURALLY_SINGULAR,
 * TOO_LARGE, OUT_OF_MEMORY, DEVICE.  Warning: NUMERICALLY_SINGULAR. */
kkt_status kkt_analyze(kkt_handle h, int32_t n, int64_t nnz, const int64_t *rowptr,
                       const int32_t *colind, const double *values0, const int32_t *user_q);

/* Re-analysis with new values for a single-system handle: the pivoting pass
 * (Section 5.1.2) re-runs on d_values (nnz(A) device doubles in the analysed
 * CSR order; copied to the host after synchronizing `stream`) with the
 * stored ordering Q, and everything is re-uploaded; the pass's factors are
 * the current factors afterwards (no kkt_refactor needed).  This is the
 * re-analysis of Section 5.1.1 for a matrix the stored pivot order no longer
 * suits.  Synchronous.
 * Errors: STATE (no single-system analysis), INVALID_ARG, as kkt_analyze. */
kkt_status kkt_reanalyze(kkt_handle h, const double *d_values, void *stream);

/* Numeric refactorization with the stored pivot sequence and patterns
 * (Section 5.1.2 "resetting the values ... and performing the
 * refactorization").  d_values: nnz(A) device doubles in the analysed CSR
 * order.  Asynchronous on `stream`; pivot health (min/max |u_kk|, tiny or
 * non-finite pivots) is recorded on the device for kkt_sync_report.
 * Errors: STATE (no analysis), INVALID_ARG, DEVICE. */
kkt_status kkt_refactor(kkt_handle h, const double *d_values, void *stream);

/* Replace the matrix the solves refine against (their residuals and Krylov
 * products) by d_values without refactorizing: the existing factors become a
 * preconditioner of a nearby matrix and FGMRES makes up the difference
 * (Section 5.1.1: the factors used like an ILU preconditioner inside the
 * Krylov method).  Asynchronous.  Errors: STATE, INVALID_ARG, DEVICE. */
kkt_status kkt_update_matrix(kkt_handle h, const double *d_values, void *stream);

/* Solve op(A) X = B with the current factors: permute, L solve, U solve,
 * permute back (Section 5.1.2), then, while eta > eta_target (or fewer than
 * min_iters iterations were done), FGMRES-CGS2 iterations preconditioned by
 * the factors, at most fgmres_max_iters per right-hand side.  op: 'N' (A) or
 * 'T' (A^T, same factors transposed).  d_b, d_x: column-major n x nrhs
 * device arrays, must not overlap.  The convergence test reads eta back to
 * the host (one small synchronous copy per right-hand side and iteration).
 * Returns KKT_OK or KKT_WARN_NOT_CONVERGED; errors STATE, INVALID_ARG,
 * DEVICE. */
kkt_status kkt_solve(kkt_handle h, char op, int32_t nrhs, const double *d_b, double *d_x,
                     void *stream);

/* Adjoint of x_r = A^{-1} b_r on the stored pattern: d_grad[p] =
 * -sum_r d_lambda[r][i] * d_x[r][j] for every stored entry p = (i,j) of A,
 * CSR order (the reverse-mode rule for a linear solve restricted to the
 * pattern).  d_lambda, d_x: column-major n x nrhs device arrays.  Async.
 * Errors: STATE, INVALID_ARG, DEVICE. */
kkt_status kkt_grad_values(kkt_handle h, int32_t nrhs, const double *d_lambda, const double *d_x,
                           double *d_grad, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): kkt_solve
 * with the device-checked refinement (whatever refine_sync says; no
 * auto_reanalyze), whose per-call scratch -- the stop-test state, reduction
 * tickets, partial sums and least-squares arrays, at most 2 MiB for restart
 * lengths up to 30 -- lives in a static device array of the library instead
 * of the handle's workspace.  It calls no allocating routine.  The handle's
 * analysis workspaces (factors, Krylov vectors) are used as by kkt_solve.
 * Every call on one GPU shares that GPU's array (the state is reset at the
 * start of each call), so calls that overlap on one GPU -- from several host
 * threads or streams -- race.  Same arguments, results and errors as
 * kkt_solve; KKT_ERR_INVALID_ARG if the refinement state does not fit the
 * array. */
kkt_status kkt_solve_noalloc(kkt_handle h, char op, int32_t nrhs, const double *d_b, double *d_x,
                             void *stream);

/* Batch of independent instances (scenarios, contingencies) solved as one
 * block-diagonal system in shared launches.  npat distinct patterns, pattern
 * p given by n[p], nnz[p], rowptr[p], colind[p] and its first values
 * values0[p]; instance t uses pattern inst_pattern[t] (count instances) and
 * reuses that pattern's ordering, pivot sequence and factor pattern, the
 * refactorization premise of Sections 4 and 5.1.  Patterns are analysed in
 * parallel host threads.  Afterwards the handle works on the concatenation:
 * kkt_refactor takes all instances' values back to back (CSR order of each),
 * kkt_solve / kkt_graph_* take all right-hand sides back to back, and eta is
 * judged per instance (kkt_batch_eta).  Errors as kkt_analyze. */
kkt_status kkt_analyze_batch(kkt_handle h, int32_t npat, const int32_t *n, const int64_t *nnz,
                             const int64_t *const *rowptr, const int32_t *const *colind,
                             const double *const *values0, int32_t count,
                             const int32_t *inst_pattern);
/* Batch of count instances of ONE pattern (n, nnz, rowptr, colind) sharing a
 * single analysis: the ordering and pivot sequence come from values0 (the
 * refactorization premise of Sections 4 and 5.1), and every index structure
 * and schedule is held once on the device while each instance has its own
 * values and vectors.  The refactorization and solve launches hand out each
 * chunk of the shared schedule once per instance.  Afterwards the handle works
 * as a block-diagonal batch of count identical patterns: kkt_refactor takes
 * count x nnz values back to back, kkt_solve / kkt_graph_* take count x n
 * right-hand sides back to back (one right-hand side per instance), eta is
 * judged per instance (kkt_batch_eta), and kkt_get_lu / kkt_get_perm /
 * kkt_get_info / kkt_batch_layout answer in that block-diagonal form.  Needs
 * the default dependency-driven kernels (matching, level-synchronous
 * schedules, the fence protocol, the kernel-variant switches, Jacobi sweeps and
 * refine_sync = 1 are rejected with INVALID_ARG, as is a pattern those kernels
 * cannot take); kkt_grad_values and kkt_solve_noalloc return STATE.  Errors
 * otherwise as kkt_analyze, plus TOO_LARGE when the batch's totals exceed the
 * int32 index range. */
kkt_status kkt_analyze_shared(kkt_handle h, int32_t n, int64_t nnz, const int64_t *rowptr,
                              const int32_t *colind, const double *values0, int32_t count);

/* Instance offsets of a batch: row_offset[count+1] into vectors,
 * nnz_offset[count+1] into the concatenated values (either may be NULL). */
kkt_status kkt_batch_layout(kkt_handle h, int64_t *row_offset, int64_t *nnz_offset);
/* eta of every instance after the last solve or graph replay (count
 * entries); synchronises. */
kkt_status kkt_batch_eta(kkt_handle h, double *eta);

/* Capture refactor(d_values) + direct solve (d_b -> d_x) + the residual check
 * into a HIP graph on `stream` (not the legacy default stream); every
 * scheduling counter lives on the device, so replays are independent.  The
 * graph has no host synchronisation and no refinement: after a replay,
 * kkt_sync_report / kkt_batch_eta give eta, and kkt_solve refines if needed.
 * The buffers must stay allocated while the graph exists; new values and
 * right-hand sides are written into the same buffers between replays.
 * Errors: STATE, INVALID_ARG, DEVICE. */
kkt_status kkt_graph_capture(kkt_handle h, const double *d_values, const double *d_b,
                             double *d_x, void *stream);
kkt_status kkt_graph_launch(kkt_handle h, void *stream);

/* Wait for the handle's device work and return (then clear) the report.  Returns
 * KKT_ERR_DEVICE if a dependency wait gave up (results invalid), KKT_ERR_NONFINITE (with *out
 * filled in) if the last refactorization's values held a NaN or an infinity. */
kkt_status kkt_sync_report(kkt_handle h, kkt_report *out);
kkt_status kkt_get_info(kkt_handle h, kkt_info *out);

/* Host copies of the permutations (n entries each; either may be NULL).
 * With matching they are those of Ahat (kkt_get_scaling). */
kkt_status kkt_get_perm(kkt_handle h, int32_t *p, int32_t *q);

/* The matching and scaling of an analysis with opt.matching = 1 (n entries
 * each; any may be NULL): match[j] = row of A placed at row j of Ahat, which
 * is scaled by dr[match[j]]; column c is scaled by dc[c].  KKT_ERR_STATE
 * without matching (Section 5.2.1). */
kkt_status kkt_get_scaling(kkt_handle h, int32_t *match, double *dr, double *dc);

/* Host copy of the current factors as one CSR matrix in pivot order: row i
 * holds L(i, 0..i-1), then u_ii, then U(i, i+1..), columns ascending.
 * rowptr: n+1, colind/values: nnz_l + nnz_u.  values may be NULL (pattern
 * only).  Synchronises the handle's device work. */
kkt_status kkt_get_lu(kkt_handle h, int64_t *rowptr, int32_t *colind, double *values);

/* Message of the last error on this handle (never NULL; "" if none). */
const char *kkt_last_error(kkt_handle h);

/* Host-only analysis (no device is touched): the exact analysis kkt_analyze
 * performs (Sections 4 and 5.1: ordering, pivot sequence, factor patterns
 * and the first factorization's values), returned as a host object for
 * inspection.  Arguments as for kkt_analyze; opt may be NULL.  On error *out
 * is NULL and, if msg is non-NULL, a message of at most msg_len bytes
 * (NUL-terminated) is written to it. */
typedef struct kkt_host_analysis *kkt_analysis;
kkt_status kkt_analysis_create(const kkt_options *opt, int32_t n, int64_t nnz,
                               const int64_t *rowptr, const int32_t *colind,
                               const double *values0, const int32_t *user_q, kkt_analysis *out,
                               char *msg, int32_t msg_len);
/* Profiling (debug_timeline = 1): the row timeline of the last refactorization, 4 values per
 * row into out (n x 4 int64, host memory): start, last poll that found an input missing, end
 * (nanoseconds from the earliest start) and the kernel (1 micro row taken by one lane, 2
 * short-row list kernel, 3 long-row kernel); rows the two band kernels did not take (rows
 * without pivots, the dense block's own steps) read -1, -1, -1, 0.  Synchronises the device.
 * Errors: INVALID_ARG, STATE (no timeline on this handle), DEVICE. */
kkt_status kkt_debug_timeline(kkt_handle h, int64_t *out);

/* Sizes and depths (device_bytes, analyze_seconds and solve_block_levels are 0; no dense
 * block is chosen, so levels_sparse equals levels). */
kkt_status kkt_analysis_info(kkt_analysis a, kkt_info *out);
/* As kkt_get_perm / kkt_get_lu, from the host object (values: the pivoting
 * pass's factors of values0). */
kkt_status kkt_analysis_perm(kkt_analysis a, int32_t *p, int32_t *q);
kkt_status kkt_analysis_scaling(kkt_analysis a, int32_t *match, double *dr, double *dc);
kkt_status kkt_analysis_lu(kkt_analysis a, int64_t *rowptr, int32_t *colind, double *values);
/* Row dependency schedule: level_ptr (levels+1 entries) and rows (n entries,
 * grouped by level); either may be NULL. */
kkt_status kkt_analysis_levels(kkt_analysis a, int32_t *level_ptr, int32_t *rows);
void kkt_analysis_destroy(kkt_analysis a);

#ifdef __cplusplus
}
#endif
#endif /* KKT_LU_H */
