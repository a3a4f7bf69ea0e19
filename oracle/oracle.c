/*
 * CPU FP64 oracle: ordering, pivoting LU, refactorization, solve with
 * FGMRES-CGS2 refinement, adjoint gradient.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product library.
 *
 * Every routine is the plain sequential definition of the step it names.
 * Arithmetic policy: every update is fma(-l, u, a) and divisions are IEEE
 * correctly rounded (build with -ffp-contract=off), so an independent code
 * that applies the same updates to each entry in the same (ascending pivot
 * step) order reproduces these factors bit for bit.
 *
 * parity unpinned: none.  Every exported function is named in a CPU test
 * that checks it against dense LAPACK, brute force, a closed form or an
 * invariant (the oracle pin tests).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* small growable arrays                                               */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t *a;
  int64_t len, cap;
} ivec;
typedef struct {
  double *a;
  int64_t len, cap;
} dvec;

static void ivec_push(ivec *v, int32_t x) {
  if (v->len == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 8;
    v->a = (int32_t *)realloc(v->a, (size_t)v->cap * sizeof(int32_t));
  }
  v->a[v->len++] = x;
}
static void dvec_push(dvec *v, double x) {
  if (v->len == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 8;
    v->a = (double *)realloc(v->a, (size_t)v->cap * sizeof(double));
  }
  v->a[v->len++] = x;
}
static int cmp_i32(const void *x, const void *y) {
  int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
  return (a > b) - (a < b);
}

/* ------------------------------------------------------------------ */
/* binary min-heap of (key1, key2) pairs, lexicographic                */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t *k1;
  int32_t *k2;
  int64_t len, cap;
} heap;
static int heap_less(const heap *h, int64_t i, int64_t j) {
  return h->k1[i] < h->k1[j] || (h->k1[i] == h->k1[j] && h->k2[i] < h->k2[j]);
}
static void heap_swap(heap *h, int64_t i, int64_t j) {
  int64_t t1 = h->k1[i];
  int32_t t2 = h->k2[i];
  h->k1[i] = h->k1[j];
  h->k2[i] = h->k2[j];
  h->k1[j] = t1;
  h->k2[j] = t2;
}
static void heap_push(heap *h, int64_t a, int32_t b) {
  if (h->len == h->cap) {
    h->cap = h->cap ? 2 * h->cap : 64;
    h->k1 = (int64_t *)realloc(h->k1, (size_t)h->cap * sizeof(int64_t));
    h->k2 = (int32_t *)realloc(h->k2, (size_t)h->cap * sizeof(int32_t));
  }
  int64_t i = h->len++;
  h->k1[i] = a;
  h->k2[i] = b;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (!heap_less(h, i, p)) break;
    heap_swap(h, i, p);
    i = p;
  }
}
static void heap_pop(heap *h, int64_t *a, int32_t *b) {
  *a = h->k1[0];
  *b = h->k2[0];
  h->len--;
  h->k1[0] = h->k1[h->len];
  h->k2[0] = h->k2[h->len];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, s = i;
    if (l < h->len && heap_less(h, l, s)) s = l;
    if (r < h->len && heap_less(h, r, s)) s = r;
    if (s == i) break;
    heap_swap(h, i, s);
    i = s;
  }
}
static void heap_free(heap *h) {
  free(h->k1);
  free(h->k2);
  memset(h, 0, sizeof(*h));
}

static int check_csr(int32_t n, const int64_t *rowptr, const int32_t *colind) {
  if (n < 0 || !rowptr || (n > 0 && !colind)) return 0;
  if (rowptr[0] != 0) return 0;
  for (int32_t i = 0; i < n; i++) {
    if (rowptr[i + 1] < rowptr[i]) return 0;
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++)
      if (colind[p] < 0 || colind[p] >= n) return 0;
  }
  return 1;
}

/* ------------------------------------------------------------------ */
/* Maximum-product matching and scaling (the MC64-style preprocessing   */
/* of Section 5.2.1, run before the fill-reducing ordering).            */
/*                                                                      */
/* Costs c_ij = log(cmax_j) - log|a_ij| >= 0 over the stored nonzero    */
/* entries (cmax_j = max_i |a_ij|); the perfect matching of minimum     */
/* total cost maximises the product of the matched magnitudes.  It is   */
/* found by the textbook dense Hungarian method with shortest           */
/* augmenting paths (absent entries cost +inf).  With the matching      */
/* fixed, the column potentials are the largest v <= 0 that keep        */
/* u_i + v_j <= c_ij with equality on the matching, where u_i =          */
/* c_{i,s(i)} - v_{s(i)}: shortest distances from a source joined to     */
/* every column, over edges s(i) -> j of weight c_ij - c_{i,s(i)} for     */
/* each stored (i, j), by Bellman-Ford.  Scaling by powers of two        */
/* (exact in floating point): dr_i = 2^round(u_i / ln 2), dc_j =          */
/* 2^round((v_j - log cmax_j) / ln 2), so |dr_i a_ij dc_j| <= 2 and the    */
/* matched entries lie in [1/2, 2].                                      */
/* Output: match[j] = row matched to column j.  Returns ORA_OK, or       */
/* ORA_ERR_STRUCT_SINGULAR when no perfect matching of nonzeros exists.  */
/* ------------------------------------------------------------------ */
int oracle_match_scale(int32_t n, const int64_t *rowptr, const int32_t *colind, const double *val,
                       int32_t *match, double *dr, double *dc) {
  if (!check_csr(n, rowptr, colind) || !val || !match || !dr || !dc) return ORA_ERR_ARG;
  const double INF = HUGE_VAL;
  size_t N1 = (size_t)n + 1;
  double *cmax = (double *)calloc(N1, sizeof(double));
  for (int32_t i = 0; i < n; i++)
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++)
      if (fabs(val[p]) > cmax[colind[p]]) cmax[colind[p]] = fabs(val[p]);
  /* dense cost matrix, 1-based rows and columns as in the textbook form */
  double *a = (double *)malloc(N1 * N1 * sizeof(double));
  for (size_t e = 0; e < N1 * N1; e++) a[e] = INF;
  for (int32_t i = 0; i < n; i++)
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++)
      if (val[p] != 0.0) a[(size_t)(i + 1) * N1 + colind[p] + 1] = log(cmax[colind[p]]) - log(fabs(val[p]));
  double *u = (double *)calloc(N1, sizeof(double)), *v = (double *)calloc(N1, sizeof(double));
  double *minv = (double *)malloc(N1 * sizeof(double));
  int32_t *pm = (int32_t *)calloc(N1, sizeof(int32_t)), *way = (int32_t *)calloc(N1, sizeof(int32_t));
  char *used = (char *)malloc(N1);
  int st = ORA_OK;
  for (int32_t i = 1; i <= n && st == ORA_OK; i++) {
    pm[0] = i;
    int32_t j0 = 0;
    for (int32_t j = 0; j <= n; j++) {
      minv[j] = INF;
      used[j] = 0;
    }
    do {
      used[j0] = 1;
      const int32_t i0 = pm[j0];
      double delta = INF;
      int32_t j1 = -1;
      for (int32_t j = 1; j <= n; j++)
        if (!used[j]) {
          const double cur = a[(size_t)i0 * N1 + j] - u[i0] - v[j];
          if (cur < minv[j]) {
            minv[j] = cur;
            way[j] = j0;
          }
          if (minv[j] < delta) {
            delta = minv[j];
            j1 = j;
          }
        }
      if (j1 < 0 || delta == INF) {
        st = ORA_ERR_STRUCT_SINGULAR;
        break;
      }
      for (int32_t j = 0; j <= n; j++)
        if (used[j]) {
          u[pm[j]] += delta;
          v[j] -= delta;
        } else {
          minv[j] -= delta;
        }
      j0 = j1;
    } while (pm[j0] != 0);
    if (st != ORA_OK) break;
    do {
      const int32_t j1 = way[j0];
      pm[j0] = pm[j1];
      j0 = j1;
    } while (j0);
  }
  if (st == ORA_OK) {
    int32_t *scol = (int32_t *)malloc(N1 * sizeof(int32_t)); /* s(i): column of row i */
    for (int32_t j = 1; j <= n; j++) {
      match[j - 1] = pm[j] - 1;
      scol[pm[j] - 1] = j - 1;
    }
    /* canonical column potentials by Bellman-Ford from a source joined to all */
    double *d = (double *)calloc(N1, sizeof(double));
    for (int32_t pass = 0; pass <= n; pass++) {
      int changed = 0;
      for (int32_t i = 0; i < n; i++) {
        const int32_t js = scol[i];
        const double cis = a[(size_t)(i + 1) * N1 + js + 1];
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
          const int32_t j = colind[p];
          const double cij = a[(size_t)(i + 1) * N1 + j + 1];
          if (cij == INF) continue;
          const double nd = d[js] + (cij - cis);
          if (nd < d[j]) {
            d[j] = nd;
            changed = 1;
          }
        }
      }
      if (!changed) break;
    }
    const double ln2 = log(2.0);
    for (int32_t i = 0; i < n; i++) {
      const int32_t js = scol[i];
      const double ui = a[(size_t)(i + 1) * N1 + js + 1] - d[js];
      dr[i] = ldexp(1.0, (int)lround(ui / ln2));
    }
    for (int32_t j = 0; j < n; j++) dc[j] = ldexp(1.0, (int)lround((d[j] - log(cmax[j])) / ln2));
    free(d);
    free(scol);
  }
  free(cmax);
  free(a);
  free(u);
  free(v);
  free(minv);
  free(pm);
  free(way);
  free(used);
  return st;
}

/* ------------------------------------------------------------------ */
/* Ordering: exact minimum degree on the elimination graph of A + A^T  */
/* (fill-reducing symmetric ordering, Sections 5.1 and 5.2).           */
/* The elimination graph is kept explicitly: eliminating v joins all of */
/* its neighbours into a clique.  Degree = current neighbour count.     */
/* ------------------------------------------------------------------ */
int oracle_order_md(int32_t n, const int64_t *rowptr, const int32_t *colind, int32_t *Q) {
  if (!check_csr(n, rowptr, colind) || (n > 0 && !Q)) return ORA_ERR_ARG;
  ivec *adj = (ivec *)calloc((size_t)n + 1, sizeof(ivec));
  for (int32_t i = 0; i < n; i++)
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
      int32_t j = colind[p];
      if (j == i) continue;
      ivec_push(&adj[i], j);
      ivec_push(&adj[j], i);
    }
  for (int32_t i = 0; i < n; i++) { /* sort + unique */
    if (adj[i].len == 0) continue;
    qsort(adj[i].a, (size_t)adj[i].len, sizeof(int32_t), cmp_i32);
    int64_t w = 1;
    for (int64_t r = 1; r < adj[i].len; r++)
      if (adj[i].a[r] != adj[i].a[w - 1]) adj[i].a[w++] = adj[i].a[r];
    adj[i].len = w;
  }
  char *elim = (char *)calloc((size_t)n + 1, 1);
  heap h = {0};
  for (int32_t i = 0; i < n; i++) heap_push(&h, adj[i].len, i);
  ivec merged = {0};
  for (int32_t step = 0; step < n; step++) {
    int64_t d;
    int32_t v;
    for (;;) { /* discard stale heap entries */
      heap_pop(&h, &d, &v);
      if (!elim[v] && d == adj[v].len) break;
    }
    Q[step] = v;
    elim[v] = 1;
    /* every neighbour u gets adj(u) := (adj(u) U adj(v)) \ {u, v} */
    for (int64_t t = 0; t < adj[v].len; t++) {
      int32_t u = adj[v].a[t];
      merged.len = 0;
      int64_t x = 0, y = 0;
      while (x < adj[u].len || y < adj[v].len) {
        int32_t c;
        if (y >= adj[v].len || (x < adj[u].len && adj[u].a[x] < adj[v].a[y]))
          c = adj[u].a[x++];
        else if (x >= adj[u].len || adj[v].a[y] < adj[u].a[x])
          c = adj[v].a[y++];
        else {
          c = adj[u].a[x];
          x++;
          y++;
        }
        if (c != u && c != v) ivec_push(&merged, c);
      }
      ivec tmp = adj[u];
      adj[u] = merged;
      merged = tmp;
      heap_push(&h, adj[u].len, u);
    }
    free(adj[v].a);
    memset(&adj[v], 0, sizeof(ivec));
  }
  free(merged.a);
  heap_free(&h);
  free(elim);
  free(adj);
  return ORA_OK;
}

/* ------------------------------------------------------------------ */
/* factor handle                                                        */
/* ------------------------------------------------------------------ */
struct oracle_lu {
  int32_t n;
  int64_t nnz;
  int64_t *rowptr; /* A in CSR (copy) */
  int32_t *colind;
  double *aval;
  int64_t *cp; /* A in CSC: column pointers, row indices, CSR position */
  int32_t *ci;
  int64_t *cpos;
  int32_t *Q, *Qinv, *P, *Pinv;
  int64_t *Lp, *Up; /* CSC, pivot order; U's diagonal last in its column */
  int32_t *Li, *Ui;
  double *Lx, *Ux;
  double anorm_inf, anorm_one;
};

void oracle_lu_free(oracle_lu *lu) {
  if (!lu) return;
  free(lu->rowptr);
  free(lu->colind);
  free(lu->aval);
  free(lu->cp);
  free(lu->ci);
  free(lu->cpos);
  free(lu->Q);
  free(lu->Qinv);
  free(lu->P);
  free(lu->Pinv);
  free(lu->Lp);
  free(lu->Up);
  free(lu->Li);
  free(lu->Ui);
  free(lu->Lx);
  free(lu->Ux);
  free(lu);
}

static void set_values(oracle_lu *lu, const double *val) {
  memcpy(lu->aval, val, (size_t)lu->nnz * sizeof(double));
  double ninf = 0.0;
  double *colsum = (double *)calloc((size_t)lu->n + 1, sizeof(double));
  for (int32_t i = 0; i < lu->n; i++) {
    double s = 0.0;
    for (int64_t p = lu->rowptr[i]; p < lu->rowptr[i + 1]; p++) {
      s += fabs(val[p]);
      colsum[lu->colind[p]] += fabs(val[p]);
    }
    if (s > ninf) ninf = s;
  }
  double none = 0.0;
  for (int32_t j = 0; j < lu->n; j++)
    if (colsum[j] > none) none = colsum[j];
  free(colsum);
  lu->anorm_inf = ninf;
  lu->anorm_one = none;
}

/* Gilbert-Peierls left-looking LU with threshold partial pivoting.
 * Column k of A' is x := A'(:,k); every earlier pivot step j whose pivot row
 * is structurally present in x is applied, in ascending j:
 *     x[r] -= L(r, j) * x[pivot row of j]   for r in L(:,j).
 * A min-heap over pivot steps yields them in ascending order; a row entering
 * the structure through L(:,j) can only carry a pivot step larger than j, so
 * the heap never needs a step smaller than the one just popped.
 * Pivot rule: the diagonal candidate (A'-row k) if |x_d| >= tau * max|x| and
 * x_d != 0, else the largest |x| (ties: smallest A'-row); if all candidates
 * are zero, the diagonal candidate (else the smallest one) and a warning, as
 * the factorization continues on singular input (Section 5.1.2). */
oracle_lu *oracle_factor(int32_t n, const int64_t *rowptr, const int32_t *colind,
                         const double *val, const int32_t *Q, double tau, int *status) {
  int st = ORA_OK;
  if (status) *status = ORA_ERR_ARG;
  if (!check_csr(n, rowptr, colind) || !Q || !val || !(tau > 0.0 && tau <= 1.0)) return NULL;
  oracle_lu *lu = (oracle_lu *)calloc(1, sizeof(oracle_lu));
  lu->n = n;
  lu->nnz = rowptr[n];
  size_t N1 = (size_t)n + 1, NZ = (size_t)lu->nnz + 1;
  lu->rowptr = (int64_t *)malloc(N1 * sizeof(int64_t));
  lu->colind = (int32_t *)malloc(NZ * sizeof(int32_t));
  lu->aval = (double *)malloc(NZ * sizeof(double));
  memcpy(lu->rowptr, rowptr, N1 * sizeof(int64_t));
  memcpy(lu->colind, colind, (size_t)lu->nnz * sizeof(int32_t));
  /* CSC of A */
  lu->cp = (int64_t *)calloc(N1 + 1, sizeof(int64_t));
  lu->ci = (int32_t *)malloc(NZ * sizeof(int32_t));
  lu->cpos = (int64_t *)malloc(NZ * sizeof(int64_t));
  for (int64_t p = 0; p < lu->nnz; p++) lu->cp[colind[p] + 1]++;
  for (int32_t j = 0; j < n; j++) lu->cp[j + 1] += lu->cp[j];
  int64_t *fillc = (int64_t *)malloc(N1 * sizeof(int64_t));
  memcpy(fillc, lu->cp, N1 * sizeof(int64_t));
  for (int32_t i = 0; i < n; i++)
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
      int64_t q = fillc[colind[p]]++;
      lu->ci[q] = i;
      lu->cpos[q] = p;
    }
  free(fillc);
  lu->Q = (int32_t *)malloc(N1 * sizeof(int32_t));
  lu->Qinv = (int32_t *)malloc(N1 * sizeof(int32_t));
  lu->P = (int32_t *)malloc(N1 * sizeof(int32_t));
  lu->Pinv = (int32_t *)malloc(N1 * sizeof(int32_t));
  for (int32_t k = 0; k < n; k++) lu->Qinv[k] = -1;
  for (int32_t k = 0; k < n; k++) {
    if (Q[k] < 0 || Q[k] >= n || lu->Qinv[Q[k]] >= 0) {
      oracle_lu_free(lu);
      return NULL;
    }
    lu->Q[k] = Q[k];
    lu->Qinv[Q[k]] = k;
  }
  set_values(lu, val);

  /* factor columns; L rows are recorded as A'-rows and renumbered at the end */
  double *x = (double *)calloc(N1, sizeof(double));
  char *inS = (char *)calloc(N1, 1);
  int32_t *pivstep = (int32_t *)malloc(N1 * sizeof(int32_t)); /* A'-row -> step */
  for (int32_t r = 0; r < n; r++) pivstep[r] = -1;
  ivec S = {0}; /* structure of x (A'-rows) */
  ivec Li = {0}, Ui = {0};
  dvec Lx = {0}, Ux = {0};
  int64_t *Lp = (int64_t *)calloc(N1, sizeof(int64_t));
  int64_t *Up = (int64_t *)calloc(N1, sizeof(int64_t));
  heap h = {0};
  for (int32_t k = 0; k < n; k++) {
    int32_t c = Q[k]; /* column of A holding A'(:,k) */
    S.len = 0;
    for (int64_t q = lu->cp[c]; q < lu->cp[c + 1]; q++) {
      int32_t r = lu->Qinv[lu->ci[q]];
      x[r] = val[lu->cpos[q]];
      inS[r] = 1;
      ivec_push(&S, r);
      if (pivstep[r] >= 0) heap_push(&h, pivstep[r], r);
    }
    /* ascending pivot steps; U(:,k) strict part = popped steps */
    int64_t u_start = Ui.len;
    while (h.len > 0) {
      int64_t j;
      int32_t prow;
      heap_pop(&h, &j, &prow);
      double xj = x[prow];
      ivec_push(&Ui, (int32_t)j);
      dvec_push(&Ux, xj);
      for (int64_t t = Lp[j]; t < Lp[j + 1]; t++) {
        int32_t r = Li.a[t];
        if (!inS[r]) {
          inS[r] = 1;
          x[r] = 0.0;
          ivec_push(&S, r);
          if (pivstep[r] >= 0) heap_push(&h, pivstep[r], r);
        }
        x[r] = fma(-Lx.a[t], xj, x[r]);
      }
    }
    (void)u_start;
    /* pivot choice among the candidates (structurally present, not yet pivotal) */
    double amax = 0.0;
    int32_t amax_row = -1, first_cand = -1;
    int has_diag = 0;
    for (int64_t t = 0; t < S.len; t++) {
      int32_t r = S.a[t];
      if (pivstep[r] >= 0) continue;
      if (r == k) has_diag = 1;
      if (first_cand < 0 || r < first_cand) first_cand = r;
      double ax = fabs(x[r]);
      if (amax_row < 0 || ax > amax || (ax == amax && r < amax_row)) {
        amax = ax;
        amax_row = r;
      }
    }
    int32_t piv;
    if (first_cand < 0) {
      st = ORA_ERR_STRUCT_SINGULAR;
      for (int64_t t = 0; t < S.len; t++) inS[S.a[t]] = 0;
      break;
    }
    if (amax == 0.0) {
      piv = has_diag ? k : first_cand;
      if (st == ORA_OK) st = ORA_WARN_SINGULAR;
    } else if (has_diag && fabs(x[k]) >= tau * amax && x[k] != 0.0) {
      piv = k;
    } else {
      piv = amax_row;
    }
    double pv = x[piv];
    ivec_push(&Ui, k);
    dvec_push(&Ux, pv);
    Up[k + 1] = Ui.len;
    pivstep[piv] = k;
    lu->P[k] = piv;
    for (int64_t t = 0; t < S.len; t++) {
      int32_t r = S.a[t];
      if (pivstep[r] < 0) {
        ivec_push(&Li, r);
        dvec_push(&Lx, x[r] / pv);
      }
      inS[r] = 0;
      x[r] = 0.0;
    }
    Lp[k + 1] = Li.len;
  }
  heap_free(&h);
  free(S.a);
  free(x);
  free(inS);
  if (st == ORA_ERR_STRUCT_SINGULAR) {
    free(pivstep);
    free(Li.a);
    free(Ui.a);
    free(Lx.a);
    free(Ux.a);
    free(Lp);
    free(Up);
    oracle_lu_free(lu);
    if (status) *status = st;
    return NULL;
  }
  /* renumber L rows into pivot order and sort each column */
  for (int32_t k = 0; k < n; k++) lu->Pinv[lu->P[k]] = k;
  for (int64_t t = 0; t < Li.len; t++) Li.a[t] = pivstep[Li.a[t]];
  for (int32_t k = 0; k < n; k++) { /* insertion sort keeps (row, value) pairs */
    for (int64_t a = Lp[k] + 1; a < Lp[k + 1]; a++) {
      int32_t r = Li.a[a];
      double v = Lx.a[a];
      int64_t b = a - 1;
      while (b >= Lp[k] && Li.a[b] > r) {
        Li.a[b + 1] = Li.a[b];
        Lx.a[b + 1] = Lx.a[b];
        b--;
      }
      Li.a[b + 1] = r;
      Lx.a[b + 1] = v;
    }
  }
  free(pivstep);
  lu->Lp = Lp;
  lu->Up = Up;
  lu->Li = Li.a ? Li.a : (int32_t *)malloc(4);
  lu->Lx = Lx.a ? Lx.a : (double *)malloc(8);
  lu->Ui = Ui.a ? Ui.a : (int32_t *)malloc(4);
  lu->Ux = Ux.a ? Ux.a : (double *)malloc(8);
  if (status) *status = st;
  return lu;
}

void oracle_lu_sizes(const oracle_lu *lu, int64_t *lnz, int64_t *unz) {
  if (lnz) *lnz = lu->Lp[lu->n];
  if (unz) *unz = lu->Up[lu->n];
}

void oracle_lu_export(const oracle_lu *lu, int32_t *P, int32_t *Q, int64_t *Lp, int32_t *Li,
                      double *Lx, int64_t *Up, int32_t *Ui, double *Ux) {
  int32_t n = lu->n;
  int64_t lnz = lu->Lp[n], unz = lu->Up[n];
  if (P) memcpy(P, lu->P, (size_t)n * sizeof(int32_t));
  if (Q) memcpy(Q, lu->Q, (size_t)n * sizeof(int32_t));
  if (Lp) memcpy(Lp, lu->Lp, ((size_t)n + 1) * sizeof(int64_t));
  if (Up) memcpy(Up, lu->Up, ((size_t)n + 1) * sizeof(int64_t));
  if (Li) memcpy(Li, lu->Li, (size_t)lnz * sizeof(int32_t));
  if (Lx) memcpy(Lx, lu->Lx, (size_t)lnz * sizeof(double));
  if (Ui) memcpy(Ui, lu->Ui, (size_t)unz * sizeof(int32_t));
  if (Ux) memcpy(Ux, lu->Ux, (size_t)unz * sizeof(double));
}

/* (|L||U|)_ij = sum_k |l_ik| |u_kj| over the pattern, k <= min(i,j), l_ii = 1. */
void oracle_lu_absprod(const oracle_lu *lu, double *sL, double *sU) {
  int32_t n = lu->n;
  double *w = (double *)calloc((size_t)n + 1, sizeof(double));
  for (int32_t j = 0; j < n; j++) {
    /* column j of |L||U| = sum_k |u_kj| * |L(:,k)| (with unit diagonal) */
    for (int64_t t = lu->Up[j]; t < lu->Up[j + 1]; t++) {
      int32_t k = lu->Ui[t];
      double u = fabs(lu->Ux[t]);
      w[k] += u;
      for (int64_t s = lu->Lp[k]; s < lu->Lp[k + 1]; s++) w[lu->Li[s]] += fabs(lu->Lx[s]) * u;
    }
    for (int64_t t = lu->Up[j]; t < lu->Up[j + 1]; t++) sU[t] = w[lu->Ui[t]];
    for (int64_t s = lu->Lp[j]; s < lu->Lp[j + 1]; s++) sL[s] = w[lu->Li[s]];
    for (int64_t t = lu->Up[j]; t < lu->Up[j + 1]; t++) {
      int32_t k = lu->Ui[t];
      w[k] = 0.0;
      for (int64_t s = lu->Lp[k]; s < lu->Lp[k + 1]; s++) w[lu->Li[s]] = 0.0;
    }
  }
  free(w);
}

/* Growth figure of the current factors: max |u_ij| over every stored entry
 * of U (diagonal included) divided by ||A||_inf, the ratio a threshold-
 * pivoting code watches to decide that its pivot sequence has gone bad
 * (Section 5.1.1: re-analysis when the solution quality degrades). */
double oracle_lu_growth(const oracle_lu *lu) {
  double umax = 0.0;
  for (int64_t t = 0; t < lu->Up[lu->n]; t++)
    if (!(fabs(lu->Ux[t]) <= umax)) umax = fabs(lu->Ux[t]);
  return lu->anorm_inf > 0.0 ? umax / lu->anorm_inf : (umax > 0.0 ? INFINITY : 0.0);
}

/* Replace the matrix used by the solves' residuals without refactoring
 * (gives a stale preconditioner for refinement tests). */
int oracle_set_values(oracle_lu *lu, const double *val) {
  if (!lu || !val) return ORA_ERR_ARG;
  set_values(lu, val);
  return ORA_OK;
}

/* Refactorization with the stored pivot sequence and patterns (Section 5.1.2,
 * "resetting the values ... using the prior pivot sequence").  Column k:
 * scatter A'(:,k) into pivot-order work w, then for j in U(:,k), j < k,
 * ascending: w[i] -= L(i,j) * w[j] for i in L(:,j); u_kk = w[k];
 * L(:,k) = w / u_kk.  A pivot with |u_kk| < tiny_rel * ||A||_inf (or a
 * non-finite one) raises the tiny-pivot warning; the factorization goes on. */
int oracle_refactor(oracle_lu *lu, const double *val, double tiny_rel) {
  return oracle_refactor_perturbed(lu, val, tiny_rel, 0.0);
}

/* The same with static pivoting: a finite pivot with |u_kk| below
 * perturb_rel * ||A||_inf is replaced by that threshold with the pivot's sign
 * (copysign) before the column of L is formed; the return value is then
 * ORA_WARN_PERTURBED (the tiny-pivot test applies to the pivots used). */
int oracle_refactor_perturbed(oracle_lu *lu, const double *val, double tiny_rel,
                              double perturb_rel) {
  if (!lu || !val) return ORA_ERR_ARG;
  int32_t n = lu->n;
  set_values(lu, val);
  double *w = (double *)calloc((size_t)n + 1, sizeof(double));
  int st = ORA_OK, perturbed = 0;
  double tiny = tiny_rel * lu->anorm_inf;
  double thr = perturb_rel * lu->anorm_inf;
  for (int32_t k = 0; k < n; k++) {
    int32_t c = lu->Q[k];
    for (int64_t t = lu->Up[k]; t < lu->Up[k + 1]; t++) w[lu->Ui[t]] = 0.0;
    for (int64_t s = lu->Lp[k]; s < lu->Lp[k + 1]; s++) w[lu->Li[s]] = 0.0;
    for (int64_t q = lu->cp[c]; q < lu->cp[c + 1]; q++)
      w[lu->Pinv[lu->Qinv[lu->ci[q]]]] = val[lu->cpos[q]];
    for (int64_t t = lu->Up[k]; t < lu->Up[k + 1] - 1; t++) {
      int32_t j = lu->Ui[t];
      double wj = w[j];
      for (int64_t s = lu->Lp[j]; s < lu->Lp[j + 1]; s++)
        w[lu->Li[s]] = fma(-lu->Lx[s], wj, w[lu->Li[s]]);
    }
    double ukk = w[k];
    if (perturb_rel > 0.0 && fabs(ukk) < thr) {
      ukk = copysign(thr, ukk);
      w[k] = ukk;
      perturbed = 1;
    }
    if (!(fabs(ukk) >= tiny) && st == ORA_OK) st = ORA_WARN_TINY_PIVOT;
    for (int64_t t = lu->Up[k]; t < lu->Up[k + 1]; t++) lu->Ux[t] = w[lu->Ui[t]];
    for (int64_t s = lu->Lp[k]; s < lu->Lp[k + 1]; s++) lu->Lx[s] = w[lu->Li[s]] / ukk;
    for (int64_t t = lu->Up[k]; t < lu->Up[k + 1]; t++) w[lu->Ui[t]] = 0.0;
    for (int64_t s = lu->Lp[k]; s < lu->Lp[k + 1]; s++) w[lu->Li[s]] = 0.0;
  }
  free(w);
  if (st == ORA_OK && perturbed) st = ORA_WARN_PERTURBED;
  return st;
}

/* ------------------------------------------------------------------ */
/* solves                                                               */
/* ------------------------------------------------------------------ */
/* M^{-1} b with the conventions of the header. */
void oracle_lu_apply(const oracle_lu *lu, char op, const double *b, double *x) {
  int32_t n = lu->n;
  double *y = (double *)malloc(((size_t)n + 1) * sizeof(double));
  if (op == 'N') {
    for (int32_t i = 0; i < n; i++) y[i] = b[lu->Q[lu->P[i]]]; /* P Q^T b */
    for (int32_t j = 0; j < n; j++) /* L y = c, column oriented */
      for (int64_t s = lu->Lp[j]; s < lu->Lp[j + 1]; s++) y[lu->Li[s]] -= lu->Lx[s] * y[j];
    for (int32_t j = n - 1; j >= 0; j--) { /* U z = y, column oriented */
      y[j] /= lu->Ux[lu->Up[j + 1] - 1];
      for (int64_t t = lu->Up[j]; t < lu->Up[j + 1] - 1; t++) y[lu->Ui[t]] -= lu->Ux[t] * y[j];
    }
    for (int32_t k = 0; k < n; k++) x[lu->Q[k]] = y[k];
  } else {
    for (int32_t k = 0; k < n; k++) y[k] = b[lu->Q[k]]; /* s = Q^T g */
    for (int32_t j = 0; j < n; j++) {                    /* U^T t = s: column j of U is row j of U^T */
      double s = y[j];
      for (int64_t t = lu->Up[j]; t < lu->Up[j + 1] - 1; t++) s -= lu->Ux[t] * y[lu->Ui[t]];
      y[j] = s / lu->Ux[lu->Up[j + 1] - 1];
    }
    for (int32_t j = n - 1; j >= 0; j--) { /* L^T w = t */
      double s = y[j];
      for (int64_t t = lu->Lp[j]; t < lu->Lp[j + 1]; t++) s -= lu->Lx[t] * y[lu->Li[t]];
      y[j] = s;
    }
    for (int32_t i = 0; i < n; i++) x[lu->Q[lu->P[i]]] = y[i]; /* l = Q P^T w */
  }
  free(y);
}

/* Approximate preconditioner of the sweep-based triangular solves (Section 6
 * names iterative triangular solves as future work): with c = P Q^T b,
 * split L = I + L_s and U = D + U_s.  The L triangle takes `sweeps` Jacobi
 * sweeps y <- c - L_s y from y = c, the U triangle `sweeps` sweeps
 * z <- D^{-1} (y - U_s z) from z = y, and x = Q z.  Each sweep reads only the
 * previous iterate.  As many sweeps as the dependency depth of a triangle
 * give its exact solve (L_s and D^{-1} U_s are nilpotent). */
void oracle_lu_apply_jacobi(const oracle_lu *lu, const double *b, int32_t sweeps, double *x) {
  int32_t n = lu->n;
  size_t N = (size_t)n + 1;
  double *c = (double *)malloc(N * sizeof(double));
  double *y = (double *)malloc(N * sizeof(double));
  double *t = (double *)malloc(N * sizeof(double));
  for (int32_t i = 0; i < n; i++) c[i] = b[lu->Q[lu->P[i]]];
  memcpy(y, c, (size_t)n * sizeof(double));
  for (int32_t k = 0; k < sweeps; k++) {
    memcpy(t, c, (size_t)n * sizeof(double)); /* t = c - L_s y, column by column */
    for (int32_t j = 0; j < n; j++)
      for (int64_t s = lu->Lp[j]; s < lu->Lp[j + 1]; s++) t[lu->Li[s]] -= lu->Lx[s] * y[j];
    memcpy(y, t, (size_t)n * sizeof(double));
  }
  double *z = c; /* c is no longer needed */
  memcpy(z, y, (size_t)n * sizeof(double));
  for (int32_t k = 0; k < sweeps; k++) {
    memcpy(t, y, (size_t)n * sizeof(double)); /* t = y - U_s z */
    for (int32_t j = 0; j < n; j++)
      for (int64_t s = lu->Up[j]; s < lu->Up[j + 1] - 1; s++) t[lu->Ui[s]] -= lu->Ux[s] * z[j];
    for (int32_t j = 0; j < n; j++) z[j] = t[j] / lu->Ux[lu->Up[j + 1] - 1];
  }
  for (int32_t k = 0; k < n; k++) x[lu->Q[k]] = z[k];
  free(c);
  free(y);
  free(t);
}

/* y = op(A) x */
static void spmv(const oracle_lu *lu, char op, const double *x, double *y) {
  int32_t n = lu->n;
  if (op == 'N') {
    for (int32_t i = 0; i < n; i++) {
      double s = 0.0;
      for (int64_t p = lu->rowptr[i]; p < lu->rowptr[i + 1]; p++) s += lu->aval[p] * x[lu->colind[p]];
      y[i] = s;
    }
  } else {
    for (int32_t j = 0; j < n; j++) {
      double s = 0.0;
      for (int64_t q = lu->cp[j]; q < lu->cp[j + 1]; q++) s += lu->aval[lu->cpos[q]] * x[lu->ci[q]];
      y[j] = s;
    }
  }
}

static double norm_inf(int32_t n, const double *v) {
  double m = 0.0;
  for (int32_t i = 0; i < n; i++)
    if (fabs(v[i]) > m || isnan(v[i])) m = isnan(v[i]) ? NAN : fabs(v[i]);
  return m;
}
static double dot(int32_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int32_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

/* r = b - op(A) x, returns eta = ||r||_inf / (||op(A)||_inf ||x||_inf) */
static double residual(const oracle_lu *lu, char op, const double *b, const double *x, double *r) {
  int32_t n = lu->n;
  spmv(lu, op, x, r);
  for (int32_t i = 0; i < n; i++) r[i] = b[i] - r[i];
  double an = op == 'N' ? lu->anorm_inf : lu->anorm_one;
  double den = an * norm_inf(n, x);
  double rn = norm_inf(n, r);
  if (den == 0.0) return rn == 0.0 ? 0.0 : INFINITY;
  return rn / den;
}

/* Flexible GMRES with the LU as right preconditioner and classical
 * Gram-Schmidt applied twice (Section 5.1.2: refinement as FGMRES with
 * CGS2, factors used like an ILU preconditioner).  Restarted with length m,
 * at most max_iters iterations in total; the exit test uses the true residual
 * of the current iterate after every iteration.  One right-hand side. */
static void fgmres_one(const oracle_lu *lu, char op, const double *b, double *x,
                       const oracle_solve_opts *o, int32_t *iters_out, double *eta_out,
                       double *eta0_out) {
  int32_t n = lu->n, m = o->restart > 0 ? o->restart : 1;
  size_t N = (size_t)n + 1;
  double *r = (double *)malloc(N * sizeof(double));
  double *xt = (double *)malloc(N * sizeof(double));
  double *w = (double *)malloc(N * sizeof(double));
  double *V = (double *)malloc(N * (size_t)(m + 1) * sizeof(double));
  double *Z = (double *)malloc(N * (size_t)m * sizeof(double));
  double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double)); /* column-major */
  double *cs = (double *)malloc((size_t)m * sizeof(double));
  double *sn = (double *)malloc((size_t)m * sizeof(double));
  double *g = (double *)malloc((size_t)(m + 1) * sizeof(double));
  double *hv = (double *)malloc((size_t)(m + 1) * sizeof(double));
  double *y = (double *)malloc((size_t)(m + 1) * sizeof(double));

  oracle_lu_apply(lu, op, b, x); /* direct solve */
  double eta = residual(lu, op, b, x, r);
  *eta0_out = eta;
  int32_t it = 0;
  int done = (eta <= o->eta_target) && (it >= o->min_iters);
  while (!done && it < o->max_iters) {
    double beta = sqrt(dot(n, r, r));
    if (!(beta > 0.0)) break;
    for (int32_t i = 0; i < n; i++) V[i] = r[i] / beta;
    for (int32_t i = 0; i <= m; i++) g[i] = 0.0;
    g[0] = beta;
    int32_t j;
    for (j = 0; j < m && it < o->max_iters; j++) {
      double *vj = V + (size_t)j * N, *zj = Z + (size_t)j * N;
      oracle_lu_apply(lu, op, vj, zj);
      spmv(lu, op, zj, w);
      /* CGS2: two classical projections against v_0..v_j */
      for (int32_t i = 0; i <= j; i++) hv[i] = dot(n, V + (size_t)i * N, w);
      for (int32_t i = 0; i <= j; i++)
        for (int32_t t = 0; t < n; t++) w[t] -= hv[i] * V[(size_t)i * N + t];
      for (int32_t i = 0; i <= j; i++) {
        double h2 = dot(n, V + (size_t)i * N, w);
        y[i] = h2;
      }
      for (int32_t i = 0; i <= j; i++) {
        for (int32_t t = 0; t < n; t++) w[t] -= y[i] * V[(size_t)i * N + t];
        hv[i] += y[i];
      }
      double hn = sqrt(dot(n, w, w));
      double *Hj = H + (size_t)j * (m + 1);
      for (int32_t i = 0; i <= j; i++) Hj[i] = hv[i];
      Hj[j + 1] = hn;
      if (hn > 0.0)
        for (int32_t t = 0; t < n; t++) V[(size_t)(j + 1) * N + t] = w[t] / hn;
      /* Givens rotations: previous ones, then a new one zeroing H[j+1][j] */
      for (int32_t i = 0; i < j; i++) {
        double a = Hj[i], c = Hj[i + 1];
        Hj[i] = cs[i] * a + sn[i] * c;
        Hj[i + 1] = -sn[i] * a + cs[i] * c;
      }
      double den = hypot(Hj[j], Hj[j + 1]);
      cs[j] = den > 0.0 ? Hj[j] / den : 1.0;
      sn[j] = den > 0.0 ? Hj[j + 1] / den : 0.0;
      Hj[j] = den;
      Hj[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      it++;
      /* iterate x0 + Z y with R y = g (back substitution) */
      for (int32_t i = j; i >= 0; i--) {
        double s = g[i];
        for (int32_t t = i + 1; t <= j; t++) s -= H[(size_t)t * (m + 1) + i] * y[t];
        y[i] = s / H[(size_t)i * (m + 1) + i];
      }
      for (int32_t t = 0; t < n; t++) xt[t] = x[t];
      for (int32_t i = 0; i <= j; i++)
        for (int32_t t = 0; t < n; t++) xt[t] += y[i] * Z[(size_t)i * N + t];
      eta = residual(lu, op, b, xt, r);
      if ((eta <= o->eta_target && it >= o->min_iters) || !(hn > 0.0)) {
        done = 1;
        j++;
        break;
      }
    }
    for (int32_t t = 0; t < n; t++) x[t] = xt[t]; /* restart from the current iterate */
    if (!done) eta = residual(lu, op, b, x, r);
    if (eta <= o->eta_target && it >= o->min_iters) done = 1;
  }
  *iters_out = it;
  *eta_out = eta;
  free(r);
  free(xt);
  free(w);
  free(V);
  free(Z);
  free(H);
  free(cs);
  free(sn);
  free(g);
  free(hv);
  free(y);
}

/* Classical iterative refinement with the factors as the approximate
 * inverse (Section 5.1.1: refinement of the direct solution): after the
 * direct solve, x <- x + M^{-1} (b - A x) until the exit test of fgmres_one
 * holds or max_iters corrections were applied.  One right-hand side. */
static void ir_one(const oracle_lu *lu, char op, const double *b, double *x,
                   const oracle_solve_opts *o, int32_t *iters_out, double *eta_out,
                   double *eta0_out) {
  int32_t n = lu->n;
  size_t N = (size_t)n + 1;
  double *r = (double *)malloc(N * sizeof(double));
  double *d = (double *)malloc(N * sizeof(double));
  oracle_lu_apply(lu, op, b, x);
  double eta = residual(lu, op, b, x, r);
  *eta0_out = eta;
  int32_t it = 0;
  while (!(eta <= o->eta_target && it >= o->min_iters) && it < o->max_iters) {
    oracle_lu_apply(lu, op, r, d);
    for (int32_t t = 0; t < n; t++) x[t] += d[t];
    it++;
    eta = residual(lu, op, b, x, r);
  }
  *iters_out = it;
  *eta_out = eta;
  free(r);
  free(d);
}

int oracle_solve(const oracle_lu *lu, char op, int32_t nrhs, const double *b, double *x,
                 const oracle_solve_opts *opt, oracle_solve_info *info) {
  if (!lu || !b || !x || nrhs < 0 || (op != 'N' && op != 'T')) return ORA_ERR_ARG;
  oracle_solve_opts o = {20, 20, 0, 1e-12, 0};
  if (opt) o = *opt;
  int32_t n = lu->n, maxit = 0;
  double emax = 0.0, e0max = 0.0;
  int conv = 1;
  for (int32_t r = 0; r < nrhs; r++) {
    int32_t it;
    double eta, eta0;
    if (o.method == 1)
      ir_one(lu, op, b + (size_t)r * n, x + (size_t)r * n, &o, &it, &eta, &eta0);
    else
      fgmres_one(lu, op, b + (size_t)r * n, x + (size_t)r * n, &o, &it, &eta, &eta0);
    if (it > maxit) maxit = it;
    if (!(eta <= emax)) emax = eta;
    if (!(eta0 <= e0max)) e0max = eta0;
    if (!(eta <= o.eta_target)) conv = 0;
  }
  if (info) {
    info->iters = maxit;
    info->converged = conv;
    info->eta = emax;
    info->eta0 = e0max;
  }
  return conv ? ORA_OK : ORA_WARN_NOT_CONVERGED;
}

int oracle_fgmres_trace(const oracle_lu *lu, char prec, const double *b, int32_t iters, double *V,
                        double *Z, double *H) {
  int32_t n = lu->n;
  size_t N = (size_t)n;
  double *w = (double *)malloc((N + 1) * sizeof(double));
  double *hv = (double *)malloc(((size_t)iters + 1) * sizeof(double));
  double *h2 = (double *)malloc(((size_t)iters + 1) * sizeof(double));
  for (size_t t = 0; t < ((size_t)iters + 1) * (size_t)iters; t++) H[t] = 0.0;
  double beta = sqrt(dot(n, b, b));
  for (int32_t i = 0; i < n; i++) V[i] = b[i] / beta; /* x0 = 0, r0 = b */
  int32_t j;
  for (j = 0; j < iters; j++) {
    double *vj = V + (size_t)j * N, *zj = Z + (size_t)j * N;
    if (prec == 'L')
      oracle_lu_apply(lu, 'N', vj, zj);
    else
      memcpy(zj, vj, N * sizeof(double));
    spmv(lu, 'N', zj, w);
    for (int32_t i = 0; i <= j; i++) hv[i] = dot(n, V + (size_t)i * N, w);
    for (int32_t i = 0; i <= j; i++)
      for (int32_t t = 0; t < n; t++) w[t] -= hv[i] * V[(size_t)i * N + t];
    for (int32_t i = 0; i <= j; i++) h2[i] = dot(n, V + (size_t)i * N, w);
    for (int32_t i = 0; i <= j; i++) {
      for (int32_t t = 0; t < n; t++) w[t] -= h2[i] * V[(size_t)i * N + t];
      hv[i] += h2[i];
    }
    double hn = sqrt(dot(n, w, w));
    for (int32_t i = 0; i <= j; i++) H[(size_t)j * (iters + 1) + i] = hv[i];
    H[(size_t)j * (iters + 1) + j + 1] = hn;
    if (!(hn > 1e-300 * beta)) {
      j++;
      break;
    }
    for (int32_t t = 0; t < n; t++) V[(size_t)(j + 1) * N + t] = w[t] / hn;
  }
  free(w);
  free(hv);
  free(h2);
  return j;
}

void oracle_grad(const oracle_lu *lu, int32_t nrhs, const double *lambda, const double *x,
                 double *grad) {
  int32_t n = lu->n;
  for (int32_t i = 0; i < n; i++)
    for (int64_t p = lu->rowptr[i]; p < lu->rowptr[i + 1]; p++) {
      int32_t j = lu->colind[p];
      double s = 0.0;
      for (int32_t r = 0; r < nrhs; r++) s += lambda[(size_t)r * n + i] * x[(size_t)r * n + j];
      grad[p] = -s;
    }
}
