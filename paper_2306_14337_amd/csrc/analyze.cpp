// Host analysis: ordering, pivoting pass, factor layouts and schedules.
//
// Section 5.1 solves the first system of the sequence completely on the CPU
// (fill-reducing symmetric ordering, then an LU with pivoting that is allowed
// to continue on singular input) and extracts the permutations and the L/U
// structures for the GPU refactorization; Section 5.2 orders A + A^T the same
// way.  This file is that phase.  Arithmetic policy: every update is
// std::fma(-l, u, a), divisions are IEEE, no contraction (-ffp-contract=off),
// and the updates of each entry are applied in ascending pivot-step order, so
// the pivoting decisions depend only on the mathematical definition and not
// on traversal order.
#include "analyze.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <deque>
#include <queue>
#include <limits>
#include <set>
#include <thread>

#include "../../include/kkt_lu.h"

namespace kktlu {

int validate_csr(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colind,
                 std::string* msg) {
  if (n <= 0 || nnz < 0 || !rowptr || (nnz > 0 && !colind)) {
    if (msg) *msg = "n must be positive and rowptr/colind non-null";
    return KKT_ERR_INVALID_ARG;
  }
  if (rowptr[0] != 0 || rowptr[n] != nnz) {
    if (msg) *msg = "rowptr[0] must be 0 and rowptr[n] must equal nnz";
    return KKT_ERR_BAD_PATTERN;
  }
  for (int32_t i = 0; i < n; i++) {
    if (rowptr[i + 1] < rowptr[i]) {
      if (msg) *msg = "rowptr is not non-decreasing at row " + std::to_string(i);
      return KKT_ERR_BAD_PATTERN;
    }
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
      int32_t c = colind[p];
      if (c < 0 || c >= n) {
        if (msg) *msg = "column index out of range in row " + std::to_string(i);
        return KKT_ERR_BAD_PATTERN;
      }
      if (p > rowptr[i] && colind[p - 1] >= c) {
        if (msg) *msg = "columns unsorted or duplicated in row " + std::to_string(i);
        return KKT_ERR_BAD_PATTERN;
      }
    }
  }
  return KKT_OK;
}

// ---------------------------------------------------------------------------
// Exact minimum degree on a quotient graph.
// Variables keep a list of adjacent variables and of adjacent elements
// (eliminated vertices).  Eliminating p turns it into an element whose
// variable list is the union of its variable neighbours and of the lists of
// the elements it touches; those elements are absorbed.  The degree of a
// variable is the size of the union of its variable neighbours and its
// elements' lists, i.e. its degree in the elimination graph, recomputed
// exactly after every elimination.  Selection: smallest (degree, index).
// ---------------------------------------------------------------------------
void order_minimum_degree(int32_t n, const int64_t* rowptr, const int32_t* colind,
                          std::vector<int32_t>& Q) {
  std::vector<std::vector<int32_t>> avar(n), elist(n), lel(n);
  for (int32_t i = 0; i < n; i++)
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
      int32_t j = colind[p];
      if (j != i) {
        avar[i].push_back(j);
        avar[j].push_back(i);
      }
    }
  for (auto& a : avar) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  enum : int8_t { VAR = 0, ELEM = 1, ABSORBED = 2 };
  std::vector<int8_t> state(n, VAR);
  std::vector<int32_t> deg(n);
  std::vector<int64_t> stamp(n, 0);
  int64_t gen = 0;
  std::set<std::pair<int32_t, int32_t>> queue;
  for (int32_t v = 0; v < n; v++) {
    deg[v] = (int32_t)avar[v].size();
    queue.insert({deg[v], v});
  }
  Q.assign(n, -1);
  std::vector<int32_t> lp;
  for (int32_t step = 0; step < n; step++) {
    const int32_t p = queue.begin()->second;
    queue.erase(queue.begin());
    Q[step] = p;
    // variable list of the new element p
    gen++;
    stamp[p] = gen;
    lp.clear();
    for (int32_t u : avar[p])
      if (state[u] == VAR && stamp[u] != gen) {
        stamp[u] = gen;
        lp.push_back(u);
      }
    for (int32_t e : elist[p]) {
      if (state[e] != ELEM) continue;
      for (int32_t u : lel[e])
        if (state[u] == VAR && stamp[u] != gen) {
          stamp[u] = gen;
          lp.push_back(u);
        }
      state[e] = ABSORBED;
      std::vector<int32_t>().swap(lel[e]);
    }
    state[p] = ELEM;
    std::vector<int32_t>().swap(avar[p]);
    std::vector<int32_t>().swap(elist[p]);
    lel[p] = lp;
    const int64_t in_lp = gen;  // stamp marking lp and p
    for (int32_t v : lp) {
      auto& el = elist[v];
      el.erase(std::remove_if(el.begin(), el.end(), [&](int32_t e) { return state[e] != ELEM; }),
               el.end());
      el.push_back(p);
      auto& av = avar[v];
      av.erase(std::remove_if(av.begin(), av.end(),
                              [&](int32_t u) { return state[u] != VAR || stamp[u] == in_lp; }),
               av.end());
    }
    for (int32_t v : lp) {
      gen++;
      stamp[v] = gen;
      int32_t d = 0;
      for (int32_t u : avar[v])
        if (stamp[u] != gen) {
          stamp[u] = gen;
          d++;
        }
      for (int32_t e : elist[v])
        for (int32_t u : lel[e])
          if (stamp[u] != gen) {
            stamp[u] = gen;
            d++;
          }
      if (d != deg[v]) {
        queue.erase({deg[v], v});
        deg[v] = d;
        queue.insert({d, v});
      }
    }
  }
}

namespace {

struct ColumnFactors {
  // column-wise factors; L rows as A'-rows until renumbered
  std::vector<int64_t> lp, up;
  std::vector<int32_t> li, ui;
  std::vector<double> lx, ux;
};

// Left-looking LU of A' with threshold partial pivoting (Gilbert-Peierls):
// structure of column k by depth-first search through the columns of L
// already computed, numeric updates in ascending pivot-step order.
int pivoting_pass(int32_t n, const int64_t* rowptr, const int32_t* colind, const double* val,
                  const std::vector<int32_t>& Q, const std::vector<int32_t>& Qinv, double tau,
                  std::vector<int32_t>& P, std::vector<int32_t>& pivstep, ColumnFactors& F,
                  int* warn_singular, std::string* msg) {
  // CSC of A with positions
  std::vector<int64_t> cptr(n + 1, 0);
  int64_t nnz = rowptr[n];
  for (int64_t p = 0; p < nnz; p++) cptr[colind[p] + 1]++;
  for (int32_t j = 0; j < n; j++) cptr[j + 1] += cptr[j];
  std::vector<int32_t> crow(nnz);
  std::vector<double> cval(nnz);
  {
    std::vector<int64_t> next(cptr.begin(), cptr.end() - 1);
    for (int32_t i = 0; i < n; i++)
      for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
        int64_t q = next[colind[p]]++;
        crow[q] = i;
        cval[q] = val[p];
      }
  }
  P.assign(n, -1);
  pivstep.assign(n, -1);
  F.lp.assign(n + 1, 0);
  F.up.assign(n + 1, 0);
  std::vector<double> x(n, 0.0);
  std::vector<int32_t> seen(n, -1);
  std::vector<int32_t> cand, steps, stack;
  *warn_singular = 0;
  for (int32_t k = 0; k < n; k++) {
    cand.clear();
    steps.clear();
    const int32_t c = Q[k];
    // discover the structure
    for (int64_t q = cptr[c]; q < cptr[c + 1]; q++) {
      int32_t r = Qinv[crow[q]];
      if (seen[r] == k) continue;
      seen[r] = k;
      x[r] = 0.0;
      if (pivstep[r] < 0) {
        cand.push_back(r);
        continue;
      }
      stack.push_back(pivstep[r]);
      while (!stack.empty()) {
        int32_t j = stack.back();
        stack.pop_back();
        steps.push_back(j);
        for (int64_t t = F.lp[j]; t < F.lp[j + 1]; t++) {
          int32_t r2 = F.li[t];
          if (seen[r2] == k) continue;
          seen[r2] = k;
          x[r2] = 0.0;
          if (pivstep[r2] < 0)
            cand.push_back(r2);
          else
            stack.push_back(pivstep[r2]);
        }
      }
    }
    for (int64_t q = cptr[c]; q < cptr[c + 1]; q++) x[Qinv[crow[q]]] = cval[q];
    std::sort(steps.begin(), steps.end());
    for (int32_t j : steps) {
      const double xj = x[P[j]];
      F.ui.push_back(j);
      F.ux.push_back(xj);
      for (int64_t t = F.lp[j]; t < F.lp[j + 1]; t++)
        x[F.li[t]] = std::fma(-F.lx[t], xj, x[F.li[t]]);
    }
    if (cand.empty()) {
      if (msg) *msg = "structurally singular: no pivot candidate in column " + std::to_string(k);
      return KKT_ERR_STRUCTURALLY_SINGULAR;
    }
    int32_t best = -1, smallest = std::numeric_limits<int32_t>::max();
    double bestabs = -1.0;
    bool diag_ok = false;
    for (int32_t r : cand) {
      double a = std::fabs(x[r]);
      if (r == k) diag_ok = true;
      smallest = std::min(smallest, r);
      if (a > bestabs || (a == bestabs && r < best)) {
        bestabs = a;
        best = r;
      }
    }
    int32_t piv;
    if (bestabs == 0.0) {
      piv = diag_ok ? k : smallest;
      *warn_singular = 1;
    } else if (diag_ok && x[k] != 0.0 && std::fabs(x[k]) >= tau * bestabs) {
      piv = k;
    } else {
      piv = best;
    }
    const double pv = x[piv];
    F.ui.push_back(k);
    F.ux.push_back(pv);
    F.up[k + 1] = (int64_t)F.ui.size();
    P[k] = piv;
    pivstep[piv] = k;
    for (int32_t r : cand)
      if (r != piv) {
        F.li.push_back(r);
        F.lx.push_back(x[r] / pv);
      }
    F.lp[k + 1] = (int64_t)F.li.size();
  }
  return KKT_OK;
}

void levels_forward(int32_t n, const std::vector<int32_t>& ptr, const std::vector<int32_t>& idx,
                    std::vector<int32_t>& lev_ptr, std::vector<int32_t>& lev_rows, bool descending,
                    std::vector<int32_t>* level_of = nullptr) {
  // level(v) = 1 + max level(u) over predecessors idx[ptr[v]..ptr[v+1]);
  // predecessors of v are all < v (ascending) or > v (descending)
  std::vector<int32_t> lev(n, 0);
  int32_t nl = 0;
  for (int32_t s = 0; s < n; s++) {
    int32_t v = descending ? n - 1 - s : s;
    int32_t l = 0;
    for (int32_t t = ptr[v]; t < ptr[v + 1]; t++) l = std::max(l, lev[idx[t]] + 1);
    lev[v] = l;
    nl = std::max(nl, l + 1);
  }
  lev_ptr.assign(nl + 1, 0);
  for (int32_t v = 0; v < n; v++) lev_ptr[lev[v] + 1]++;
  for (int32_t l = 0; l < nl; l++) lev_ptr[l + 1] += lev_ptr[l];
  lev_rows.assign(n, 0);
  std::vector<int32_t> next(lev_ptr.begin(), lev_ptr.end() - 1);
  for (int32_t s = 0; s < n; s++) {
    int32_t v = descending ? n - 1 - s : s;
    lev_rows[next[lev[v]]++] = v;
  }
  if (level_of) *level_of = lev;
}

}  // namespace

int match_scale(int32_t n, const int64_t* rowptr, const int32_t* colind, const double* val,
                std::vector<int32_t>& match, std::vector<double>& dr, std::vector<double>& dc) {
  const double INF = std::numeric_limits<double>::infinity();
  const int64_t nnz = rowptr[n];
  std::vector<double> cmax(n, 0.0), c(nnz, INF);
  for (int64_t p = 0; p < nnz; p++) cmax[colind[p]] = std::max(cmax[colind[p]], std::fabs(val[p]));
  for (int32_t i = 0; i < n; i++)
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++)
      if (val[p] != 0.0) c[p] = std::log(cmax[colind[p]]) - std::log(std::fabs(val[p]));
  // successive shortest augmenting paths from each row; reduced costs
  // c_ij - u_i - v_j stay non-negative and are zero on the matching
  std::vector<double> u(n, INF), v(n, 0.0), dist(n, INF);
  for (int32_t i = 0; i < n; i++)
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) u[i] = std::min(u[i], c[p]);
  for (int32_t i = 0; i < n; i++)
    if (u[i] == INF) return KKT_ERR_STRUCTURALLY_SINGULAR;
  std::vector<int32_t> row_of(n, -1), col_of(n, -1), pred(n, -1);
  std::vector<char> done(n, 0);
  std::vector<int32_t> touched, settled;
  using Item = std::pair<double, int32_t>;
  for (int32_t r = 0; r < n; r++) {
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    auto relax = [&](int32_t i, double base) {
      for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
        const int32_t j = colind[p];
        if (c[p] == INF || done[j]) continue;
        const double d = base + (c[p] - u[i] - v[j]);
        if (d < dist[j]) {
          if (dist[j] == INF) touched.push_back(j);
          dist[j] = d;
          pred[j] = i;
          heap.push({d, j});
        }
      }
    };
    relax(r, 0.0);
    int32_t jend = -1;
    double D = 0.0;
    while (!heap.empty()) {
      const Item it = heap.top();
      heap.pop();
      const int32_t j = it.second;
      if (done[j] || it.first > dist[j]) continue;
      done[j] = 1;
      settled.push_back(j);
      if (row_of[j] < 0) {
        jend = j;
        D = it.first;
        break;
      }
      relax(row_of[j], it.first);
    }
    if (jend < 0) return KKT_ERR_STRUCTURALLY_SINGULAR;
    // new potentials: settled columns down, their rows and the root up, by
    // D - dist (keeps every reduced cost >= 0 and makes the path tight)
    for (int32_t j : settled) {
      const double dj = D - dist[j];
      if (j != jend) u[row_of[j]] += dj;
      v[j] -= dj;
    }
    u[r] += D;
    // augment along the predecessors
    for (int32_t j = jend;;) {
      const int32_t i = pred[j];
      const int32_t prev = col_of[i];
      row_of[j] = i;
      col_of[i] = j;
      if (i == r) break;
      j = prev;
    }
    for (int32_t j : touched) {
      dist[j] = INF;
      done[j] = 0;
      pred[j] = -1;
    }
    for (int32_t j : settled) done[j] = 0;
    touched.clear();
    settled.clear();
  }
  // canonical column potentials: shortest distances from a source joined to
  // every column over edges s(i) -> j of weight c_ij - c_{i,s(i)}
  std::vector<double> d(n, 0.0), cs(n);
  for (int32_t i = 0; i < n; i++) {
    const int32_t js = col_of[i];
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++)
      if (colind[p] == js) cs[i] = c[p];
  }
  std::deque<int32_t> queue;
  std::vector<char> inq(n, 1);
  for (int32_t j = 0; j < n; j++) queue.push_back(j);
  while (!queue.empty()) {
    const int32_t j0 = queue.front();
    queue.pop_front();
    inq[j0] = 0;
    const int32_t i = row_of[j0];
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
      if (c[p] == INF) continue;
      const int32_t j = colind[p];
      const double nd = d[j0] + (c[p] - cs[i]);
      if (nd < d[j]) {
        d[j] = nd;
        if (!inq[j]) {
          inq[j] = 1;
          queue.push_back(j);
        }
      }
    }
  }
  const double ln2 = std::log(2.0);
  match.assign(row_of.begin(), row_of.end());
  dr.assign(n, 1.0);
  dc.assign(n, 1.0);
  for (int32_t i = 0; i < n; i++)
    dr[i] = std::ldexp(1.0, (int)std::lround((cs[i] - d[col_of[i]]) / ln2));
  for (int32_t j = 0; j < n; j++)
    dc[j] = std::ldexp(1.0, (int)std::lround((d[j] - std::log(cmax[j])) / ln2));
  return KKT_OK;
}

int analyze_scaled(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colind,
                   const double* values, const std::vector<int32_t>& match,
                   const std::vector<double>& dr, const std::vector<double>& dc,
                   const int32_t* user_q, const AnalyzeOptions& opt, Analysis& A,
                   std::string* msg) {
  // Ahat: row j is A's row match[j], entries dr_i a_ij dc_j (exact: powers
  // of two), and the A position of each of its entries
  std::vector<int64_t> hrp(n + 1, 0), hsrc(nnz);
  std::vector<int32_t> hci(nnz);
  std::vector<double> hv(nnz);
  for (int32_t j = 0; j < n; j++) {
    const int32_t i = match[j];
    int64_t q = hrp[j];
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++, q++) {
      hci[q] = colind[p];
      hv[q] = dr[i] * values[p] * dc[colind[p]];
      hsrc[q] = p;
    }
    hrp[j + 1] = q;
  }
  AnalyzeOptions o2 = opt;
  o2.matching = 0;
  const int st = analyze(n, nnz, hrp.data(), hci.data(), hv.data(), user_q, o2, A, msg);
  if (st < 0) return st;
  // the value map refers to A's positions; per-entry scale of A's values
  for (auto& x : A.lu_src)
    if (x >= 0) x = (int32_t)hsrc[x];
  A.ascale.assign(nnz, 1.0);
  for (int32_t i = 0; i < n; i++)
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) A.ascale[p] = dr[i] * dc[colind[p]];
  A.match = match;
  A.dr = dr;
  A.dc = dc;
  return st;
}

int analyze(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colind,
            const double* values0, const int32_t* user_q, const AnalyzeOptions& opt, Analysis& A,
            std::string* msg) {
  int st = validate_csr(n, nnz, rowptr, colind, msg);
  if (st != KKT_OK) return st;
  if (!values0) {
    if (msg) *msg = "values0 is required (pivoting is numeric)";
    return KKT_ERR_INVALID_ARG;
  }
  if (!(opt.tau > 0.0 && opt.tau <= 1.0)) {
    if (msg) *msg = "pivot_tau must be in (0, 1]";
    return KKT_ERR_INVALID_ARG;
  }
  for (int64_t p = 0; p < nnz; p++)
    if (!std::isfinite(values0[p])) {
      if (msg) *msg = "values0 holds NaN or Inf at position " + std::to_string(p);
      return KKT_ERR_NONFINITE;
    }
  if (opt.matching == 1) {
    std::vector<int32_t> match;
    std::vector<double> dr, dc;
    st = match_scale(n, rowptr, colind, values0, match, dr, dc);
    if (st != KKT_OK) {
      if (msg) *msg = "no perfect matching of the nonzero entries (structurally singular)";
      return st;
    }
    return analyze_scaled(n, nnz, rowptr, colind, values0, match, dr, dc, user_q, opt, A, msg);
  }
  A = Analysis();
  A.n = n;
  A.nnz = nnz;
  // ordering
  if (opt.ordering == 0) {
    order_minimum_degree(n, rowptr, colind, A.Q);
  } else if (opt.ordering == 1) {
    A.Q.resize(n);
    for (int32_t i = 0; i < n; i++) A.Q[i] = i;
  } else if (opt.ordering == 2) {
    if (!user_q) {
      if (msg) *msg = "ordering 2 needs user_q";
      return KKT_ERR_INVALID_ARG;
    }
    A.Q.assign(user_q, user_q + n);
  } else {
    if (msg) *msg = "unknown ordering";
    return KKT_ERR_INVALID_ARG;
  }
  A.Qinv.assign(n, -1);
  for (int32_t k = 0; k < n; k++) {
    int32_t q = A.Q[k];
    if (q < 0 || q >= n || A.Qinv[q] >= 0) {
      if (msg) *msg = "Q is not a permutation";
      return KKT_ERR_INVALID_ARG;
    }
    A.Qinv[q] = k;
  }
  // pivoting pass
  ColumnFactors F;
  std::vector<int32_t> pivstep;
  st = pivoting_pass(n, rowptr, colind, values0, A.Q, A.Qinv, opt.tau, A.P, pivstep, F,
                     &A.warn_singular, msg);
  if (st != KKT_OK) return st;
  A.Pinv.assign(n, 0);
  for (int32_t k = 0; k < n; k++) A.Pinv[A.P[k]] = k;
  const int64_t lnz = F.lp[n], unz = F.up[n];
  if (lnz + unz > (int64_t)std::numeric_limits<int32_t>::max()) {
    if (msg) *msg = "nnz(L+U) exceeds the int32 index range";
    return KKT_ERR_TOO_LARGE;
  }
  A.nnz_l = lnz;
  A.nnz_u = unz;
  // combined CSR in pivot order
  std::vector<int32_t> cl(n, 0), cu(n, 0);
  for (int64_t t = 0; t < lnz; t++) cl[pivstep[F.li[t]]]++;
  for (int64_t t = 0; t < unz; t++) cu[F.ui[t]]++;
  A.lu_rowptr.assign(n + 1, 0);
  A.diag.assign(n, 0);
  for (int32_t i = 0; i < n; i++) A.lu_rowptr[i + 1] = A.lu_rowptr[i] + cl[i] + cu[i];
  const int64_t f = lnz + unz;
  A.lu_col.assign(f, 0);
  A.lu_val0.assign(f, 0.0);
  std::vector<int32_t> nl(n), nu(n);
  for (int32_t i = 0; i < n; i++) {
    nl[i] = A.lu_rowptr[i];
    nu[i] = A.lu_rowptr[i] + cl[i];
    A.diag[i] = nu[i];
  }
  for (int32_t k = 0; k < n; k++) {
    for (int64_t t = F.lp[k]; t < F.lp[k + 1]; t++) {
      int32_t i = pivstep[F.li[t]];
      A.lu_col[nl[i]] = k;
      A.lu_val0[nl[i]++] = F.lx[t];
    }
    for (int64_t t = F.up[k]; t < F.up[k + 1]; t++) {
      int32_t i = F.ui[t];
      A.lu_col[nu[i]] = k;
      A.lu_val0[nu[i]++] = F.ux[t];
    }
  }
  // A -> LU value map (gather form: LU position -> A position or -1)
  A.lu_src.assign(f, -1);
  for (int32_t r = 0; r < n; r++) {
    const int32_t i = A.Pinv[A.Qinv[r]];
    const int32_t* b = A.lu_col.data() + A.lu_rowptr[i];
    const int32_t* e = A.lu_col.data() + A.lu_rowptr[i + 1];
    for (int64_t p = rowptr[r]; p < rowptr[r + 1]; p++) {
      const int32_t j = A.Qinv[colind[p]];
      const int32_t* it = std::lower_bound(b, e, j);
      if (it == e || *it != j) {
        if (msg) *msg = "internal: A entry missing from the factor pattern";
        return KKT_ERR_DEVICE;
      }
      A.lu_src[it - A.lu_col.data()] = (int32_t)p;
    }
  }
  // schedules: rows of the dependency graph L(i,:) (refactorization, L solve)
  {
    std::vector<int32_t> ptr(n + 1), idx;
    idx.reserve(lnz);
    for (int32_t i = 0; i < n; i++) {
      for (int32_t q = A.lu_rowptr[i]; q < A.diag[i]; q++) idx.push_back(A.lu_col[q]);
      ptr[i + 1] = (int32_t)idx.size();
    }
    levels_forward(n, ptr, idx, A.lev_ptr, A.lev_rows, false);
    const int32_t nlev = (int32_t)A.lev_ptr.size() - 1;
    A.lev_maxlen.assign(nlev, 0);
    for (int32_t l = 0; l < nlev; l++)
      for (int32_t t = A.lev_ptr[l]; t < A.lev_ptr[l + 1]; t++) {
        int32_t i = A.lev_rows[t];
        A.lev_maxlen[l] = std::max(A.lev_maxlen[l], A.lu_rowptr[i + 1] - A.lu_rowptr[i]);
      }
    // U solve: row i needs z_j for j in U(i, >i)
    ptr.assign(n + 1, 0);
    idx.clear();
    for (int32_t i = 0; i < n; i++) {
      for (int32_t q = A.diag[i] + 1; q < A.lu_rowptr[i + 1]; q++) idx.push_back(A.lu_col[q]);
      ptr[i + 1] = (int32_t)idx.size();
    }
    levels_forward(n, ptr, idx, A.ulev_ptr, A.ulev_rows, true);
  }
  // transposed views: columns of U (rows ascending, diagonal last) and of strict L
  {
    A.ut_ptr.assign(n + 1, 0);
    A.lt_ptr.assign(n + 1, 0);
    for (int32_t i = 0; i < n; i++) {
      for (int32_t q = A.lu_rowptr[i]; q < A.diag[i]; q++) A.lt_ptr[A.lu_col[q] + 1]++;
      for (int32_t q = A.diag[i]; q < A.lu_rowptr[i + 1]; q++) A.ut_ptr[A.lu_col[q] + 1]++;
    }
    for (int32_t j = 0; j < n; j++) {
      A.lt_ptr[j + 1] += A.lt_ptr[j];
      A.ut_ptr[j + 1] += A.ut_ptr[j];
    }
    A.lt_pos.assign(lnz, 0);
    A.ut_pos.assign(unz, 0);
    std::vector<int32_t> nxl(A.lt_ptr.begin(), A.lt_ptr.end() - 1);
    std::vector<int32_t> nxu(A.ut_ptr.begin(), A.ut_ptr.end() - 1);
    for (int32_t i = 0; i < n; i++) {
      for (int32_t q = A.lu_rowptr[i]; q < A.diag[i]; q++) A.lt_pos[nxl[A.lu_col[q]]++] = q;
      for (int32_t q = A.diag[i]; q < A.lu_rowptr[i + 1]; q++) A.ut_pos[nxu[A.lu_col[q]]++] = q;
    }
    // U^T solve (ascending j): t_j needs t_i for i in U(:, j), i < j
    std::vector<int32_t> ptr(n + 1), idx;
    for (int32_t j = 0; j < n; j++) {
      for (int32_t t = A.ut_ptr[j]; t < A.ut_ptr[j + 1] - 1; t++) {
        int32_t q = A.ut_pos[t];
        int32_t i = (int32_t)(std::upper_bound(A.lu_rowptr.begin(), A.lu_rowptr.end(), q) -
                              A.lu_rowptr.begin()) - 1;
        idx.push_back(i);
      }
      ptr[j + 1] = (int32_t)idx.size();
    }
    levels_forward(n, ptr, idx, A.utlev_ptr, A.utlev_rows, false);
    // L^T solve (descending j): w_j needs w_i for i in L(:, j), i > j
    idx.clear();
    for (int32_t j = 0; j < n; j++) {
      for (int32_t t = A.lt_ptr[j]; t < A.lt_ptr[j + 1]; t++) {
        int32_t q = A.lt_pos[t];
        int32_t i = (int32_t)(std::upper_bound(A.lu_rowptr.begin(), A.lu_rowptr.end(), q) -
                              A.lu_rowptr.begin()) - 1;
        idx.push_back(i);
      }
      ptr[j + 1] = (int32_t)idx.size();
    }
    levels_forward(n, ptr, idx, A.ltlev_ptr, A.ltlev_rows, true);
  }
  return A.warn_singular ? KKT_WARN_NUMERICALLY_SINGULAR : KKT_OK;
}

}  // namespace kktlu

namespace kktlu {

int analyze_batch(int32_t npat, const int32_t* n, const int64_t* nnz,
                  const int64_t* const* rowptr, const int32_t* const* colind,
                  const double* const* values0, int32_t count, const int32_t* inst_pattern,
                  const AnalyzeOptions& opt, Analysis& out, std::vector<int64_t>& row_off,
                  std::vector<int64_t>& nnz_off, std::string* msg) {
  if (npat <= 0 || count <= 0 || !n || !nnz || !rowptr || !colind || !values0 || !inst_pattern) {
    if (msg) *msg = "batch: bad counts or null arrays";
    return KKT_ERR_INVALID_ARG;
  }
  for (int32_t t = 0; t < count; t++)
    if (inst_pattern[t] < 0 || inst_pattern[t] >= npat) {
      if (msg) *msg = "batch: inst_pattern out of range";
      return KKT_ERR_INVALID_ARG;
    }
  // one analysis per distinct pattern, patterns spread over host threads
  std::vector<Analysis> pa(npat);
  std::vector<int> pst(npat, KKT_OK);
  std::vector<std::string> pmsg(npat);
  {
    std::atomic<int> next(0);
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nth = (int)std::min<unsigned>(hw, (unsigned)npat);
    auto work = [&]() {
      for (int p = next++; p < npat; p = next++) {
        try {
          pst[p] = analyze(n[p], nnz[p], rowptr[p], colind[p], values0[p], nullptr, opt, pa[p],
                           &pmsg[p]);
        } catch (const std::bad_alloc&) {
          pst[p] = KKT_ERR_OUT_OF_MEMORY;
          pmsg[p] = "host allocation failed";
        }
      }
    };
    std::vector<std::thread> th;
    for (int k = 1; k < nth; k++) th.emplace_back(work);
    work();
    for (auto& x : th) x.join();
  }
  int warn = 0;
  for (int32_t p = 0; p < npat; p++) {
    if (pst[p] < 0) {
      if (msg) *msg = "batch pattern " + std::to_string(p) + ": " + pmsg[p];
      return pst[p];
    }
    warn |= pa[p].warn_singular;
  }
  row_off.assign(count + 1, 0);
  nnz_off.assign(count + 1, 0);
  std::vector<int64_t> f_off(count + 1, 0), l_off(count + 1, 0), u_off(count + 1, 0);
  size_t nlev = 0, nulev = 0, nutlev = 0, nltlev = 0;
  for (int32_t t = 0; t < count; t++) {
    const Analysis& a = pa[inst_pattern[t]];
    row_off[t + 1] = row_off[t] + a.n;
    nnz_off[t + 1] = nnz_off[t] + a.nnz;
    f_off[t + 1] = f_off[t] + (int64_t)a.lu_col.size();
    l_off[t + 1] = l_off[t] + a.nnz_l;
    u_off[t + 1] = u_off[t] + a.nnz_u;
    nlev = std::max(nlev, a.lev_ptr.size() - 1);
    nulev = std::max(nulev, a.ulev_ptr.size() - 1);
    nutlev = std::max(nutlev, a.utlev_ptr.size() - 1);
    nltlev = std::max(nltlev, a.ltlev_ptr.size() - 1);
  }
  const int64_t N = row_off[count], NNZ = nnz_off[count], F = f_off[count];
  const int64_t lim = std::numeric_limits<int32_t>::max();
  if (N > lim || NNZ > lim || F > lim) {
    if (msg) *msg = "batch exceeds the int32 index range";
    return KKT_ERR_TOO_LARGE;
  }
  Analysis& A = out;
  A = Analysis();
  A.n = (int32_t)N;
  A.nnz = NNZ;
  A.nnz_l = l_off[count];
  A.nnz_u = u_off[count];
  A.warn_singular = warn;
  A.Q.resize(N);
  A.Qinv.resize(N);
  A.P.resize(N);
  A.Pinv.resize(N);
  A.lu_rowptr.resize(N + 1);
  A.diag.resize(N);
  A.lu_col.resize(F);
  A.lu_val0.resize(F);
  A.lu_src.resize(F);
  A.ut_ptr.resize(N + 1);
  A.lt_ptr.resize(N + 1);
  A.ut_pos.resize(A.nnz_u);
  A.lt_pos.resize(A.nnz_l);
  for (int32_t t = 0; t < count; t++) {
    const Analysis& a = pa[inst_pattern[t]];
    const int32_t ro = (int32_t)row_off[t], fo = (int32_t)f_off[t], no = (int32_t)nnz_off[t];
    const int32_t lo = (int32_t)l_off[t], uo = (int32_t)u_off[t];
    for (int32_t k = 0; k < a.n; k++) {
      A.Q[ro + k] = ro + a.Q[k];
      A.Qinv[ro + k] = ro + a.Qinv[k];
      A.P[ro + k] = ro + a.P[k];
      A.Pinv[ro + k] = ro + a.Pinv[k];
      A.lu_rowptr[ro + k] = fo + a.lu_rowptr[k];
      A.diag[ro + k] = fo + a.diag[k];
      A.ut_ptr[ro + k] = uo + a.ut_ptr[k];
      A.lt_ptr[ro + k] = lo + a.lt_ptr[k];
    }
    for (size_t q = 0; q < a.lu_col.size(); q++) {
      A.lu_col[fo + q] = ro + a.lu_col[q];
      A.lu_val0[fo + q] = a.lu_val0[q];
      A.lu_src[fo + q] = a.lu_src[q] >= 0 ? no + a.lu_src[q] : -1;
    }
    for (size_t q = 0; q < a.ut_pos.size(); q++) A.ut_pos[uo + q] = fo + a.ut_pos[q];
    for (size_t q = 0; q < a.lt_pos.size(); q++) A.lt_pos[lo + q] = fo + a.lt_pos[q];
  }
  A.lu_rowptr[N] = (int32_t)F;
  A.ut_ptr[N] = (int32_t)A.nnz_u;
  A.lt_ptr[N] = (int32_t)A.nnz_l;
  // level schedules merged level by level (instances are independent, so the
  // depth is the largest instance depth, not the sum)
  auto merge = [&](size_t levels, std::vector<int32_t> Analysis::*ptr,
                   std::vector<int32_t> Analysis::*rows, std::vector<int32_t>& optr,
                   std::vector<int32_t>& orows) {
    optr.assign(levels + 1, 0);
    for (int32_t t = 0; t < count; t++) {
      const Analysis& a = pa[inst_pattern[t]];
      const auto& lp = a.*ptr;
      for (size_t l = 0; l + 1 < lp.size(); l++) optr[l + 1] += lp[l + 1] - lp[l];
    }
    for (size_t l = 0; l < levels; l++) optr[l + 1] += optr[l];
    orows.assign(N, 0);
    std::vector<int32_t> fill(optr.begin(), optr.end() - 1);
    for (int32_t t = 0; t < count; t++) {
      const Analysis& a = pa[inst_pattern[t]];
      const auto& lp = a.*ptr;
      const auto& lr = a.*rows;
      const int32_t ro = (int32_t)row_off[t];
      for (size_t l = 0; l + 1 < lp.size(); l++)
        for (int32_t q = lp[l]; q < lp[l + 1]; q++) orows[fill[l]++] = ro + lr[q];
    }
  };
  merge(nlev, &Analysis::lev_ptr, &Analysis::lev_rows, A.lev_ptr, A.lev_rows);
  merge(nulev, &Analysis::ulev_ptr, &Analysis::ulev_rows, A.ulev_ptr, A.ulev_rows);
  merge(nutlev, &Analysis::utlev_ptr, &Analysis::utlev_rows, A.utlev_ptr, A.utlev_rows);
  merge(nltlev, &Analysis::ltlev_ptr, &Analysis::ltlev_rows, A.ltlev_ptr, A.ltlev_rows);
  A.lev_maxlen.assign(nlev, 0);
  for (int32_t p = 0; p < npat; p++)
    for (size_t l = 0; l < pa[p].lev_maxlen.size(); l++)
      A.lev_maxlen[l] = std::max(A.lev_maxlen[l], pa[p].lev_maxlen[l]);
  return warn ? KKT_WARN_NUMERICALLY_SINGULAR : KKT_OK;
}

}  // namespace kktlu
