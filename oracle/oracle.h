/*
 * CPU FP64 oracle for the fixed-pattern sparse LU refactor/solve path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product library
 * shares no code, header or helper with it.
 *
 * Plain, slow, sequential definitions.  Conventions:
 *   Q[k]  original index of the k-th eliminated vertex; A' = Q^T A Q, i.e.
 *         A'[k][l] = A[Q[k]][Q[l]].
 *   P[k]  A'-row chosen as pivot at step k; P A' = L U, L unit lower
 *         triangular, U upper triangular, both indexed in pivot order.
 *   Solve A x = b:   c = Q^T b, y = U^{-1} L^{-1} (P c), x = Q y.
 *   Solve A^T l = g: s = Q^T g, t = U^{-T} s, w = L^{-T} t, l = Q (P^T w).
 *
 * Status codes match the product's public header numerically (so tests can
 * compare them) but are defined here independently.
 */
#ifndef KKT_ORACLE_H
#define KKT_ORACLE_H
#include <stdint.h>

#define ORA_OK 0
#define ORA_WARN_SINGULAR 1
#define ORA_WARN_TINY_PIVOT 2
#define ORA_WARN_NOT_CONVERGED 3
#define ORA_WARN_PERTURBED 4
#define ORA_ERR_ARG (-1)
#define ORA_ERR_STRUCT_SINGULAR (-3)

typedef struct oracle_lu oracle_lu;

typedef struct {
  int32_t restart;   /* FGMRES restart length m */
  int32_t max_iters; /* total FGMRES iteration budget */
  int32_t min_iters; /* always run at least this many iterations */
  double eta_target; /* exit when ||b-Ax||_inf / (||A||_inf ||x||_inf) <= target */
  int32_t method;    /* 0 FGMRES-CGS2, 1 classical iterative refinement */
} oracle_solve_opts;

typedef struct {
  int32_t iters;     /* FGMRES iterations spent (max over right-hand sides) */
  int32_t converged; /* 1 if every right-hand side met eta_target */
  double eta;        /* final eta (max over right-hand sides) */
  double eta0;       /* eta after the direct solve (max over right-hand sides) */
} oracle_solve_info;

/* Maximum-product perfect matching of the nonzero entries and power-of-two
 * row/column scaling from its canonical dual potentials (Section 5.2.1's
 * MC64-style preprocessing).  match[j] = row matched to column j; dr, dc: n
 * scale factors each, so that dr_i a_ij dc_j is at most 2 in magnitude and
 * the matched entries lie in [1/2, 2].  Dense O(n^2) memory: small systems.
 * Returns ORA_OK or ORA_ERR_STRUCT_SINGULAR (no perfect matching). */
int oracle_match_scale(int32_t n, const int64_t *rowptr, const int32_t *colind, const double *val,
                       int32_t *match, double *dr, double *dc);

/* Exact minimum degree on pattern(A + A^T) without the diagonal; ties go to
 * the smallest original index.  Writes Q[n].  Returns ORA_OK or ORA_ERR_ARG. */
int oracle_order_md(int32_t n, const int64_t *rowptr, const int32_t *colind, int32_t *Q);

/* Left-looking Gilbert-Peierls LU of A' with threshold partial pivoting
 * (tau in (0,1]).  Returns a handle (NULL on error); *status gets ORA_OK,
 * ORA_WARN_SINGULAR or ORA_ERR_STRUCT_SINGULAR. */
oracle_lu *oracle_factor(int32_t n, const int64_t *rowptr, const int32_t *colind,
                         const double *val, const int32_t *Q, double tau, int *status);
void oracle_lu_free(oracle_lu *lu);
/* nnz of strict L and of U (with diagonal) */
void oracle_lu_sizes(const oracle_lu *lu, int64_t *lnz, int64_t *unz);
/* CSC export in pivot order: L strict lower (rows ascending), U upper with
 * the diagonal last in each column.  Any pointer may be NULL. */
void oracle_lu_export(const oracle_lu *lu, int32_t *P, int32_t *Q, int64_t *Lp, int32_t *Li,
                      double *Lx, int64_t *Up, int32_t *Ui, double *Ux);
/* |L||U| on the pattern of L+U (componentwise backward-error scale).  Same
 * CSC layout as the export: sL for L entries, sU for U entries. */
void oracle_lu_absprod(const oracle_lu *lu, double *sL, double *sU);

/* max |u_ij| over U (diagonal included) / ||A||_inf of the current factors. */
double oracle_lu_growth(const oracle_lu *lu);

/* Refactor with the stored P, Q and patterns (no pivot search).  Returns
 * ORA_OK or ORA_WARN_TINY_PIVOT (|u_kk| < tiny_rel * ||A||_inf). */
int oracle_refactor(oracle_lu *lu, const double *val, double tiny_rel);
/* Refactorization with static pivoting (perturb_rel > 0): pivots with
 * |u_kk| < perturb_rel * ||A||_inf are replaced by copysign of that value.
 * Returns ORA_WARN_PERTURBED if any was. */
int oracle_refactor_perturbed(oracle_lu *lu, const double *val, double tiny_rel,
                              double perturb_rel);

/* Replace the matrix values used by residuals (factors left as they are). */
int oracle_set_values(oracle_lu *lu, const double *val);

/* Direct solve then FGMRES-CGS2 refinement with the stored factors as the
 * right preconditioner.  op 'N' solves A x = b, 'T' solves A^T x = b.
 * b, x: column-major n x nrhs. */
int oracle_solve(const oracle_lu *lu, char op, int32_t nrhs, const double *b, double *x,
                 const oracle_solve_opts *opt, oracle_solve_info *info);

/* Plain preconditioner application M^{-1} b (no refinement). */
void oracle_lu_apply(const oracle_lu *lu, char op, const double *b, double *x);

/* Approximate M^{-1} b by `sweeps` Jacobi sweeps per triangle (L from
 * y = c, then U from z = y), op 'N' only. */
void oracle_lu_apply_jacobi(const oracle_lu *lu, const double *b, int32_t sweeps, double *x);

/* FGMRES trace for invariant checks: exactly `iters` Arnoldi steps from
 * x0 = 0 on A x = b, preconditioner `prec` ('I' identity, 'L' the LU).
 * Outputs V (n x (iters+1)), Z (n x iters), H ((iters+1) x iters), all
 * column-major, H unrotated.  Returns the number of steps done (fewer on
 * breakdown). */
int oracle_fgmres_trace(const oracle_lu *lu, char prec, const double *b, int32_t iters, double *V,
                        double *Z, double *H);

/* Adjoint: grad[p] = -sum_r lambda[r][i] * x[r][j] for stored entry p=(i,j)
 * of A (CSR order); lambda, x column-major n x nrhs. */
void oracle_grad(const oracle_lu *lu, int32_t nrhs, const double *lambda, const double *x,
                 double *grad);

#endif
