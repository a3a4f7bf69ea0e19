// Host-side analysis of the first matrix of a same-pattern sequence:
// ordering, pivot sequence, factor patterns, value maps and schedules.
// (Sections 4 and 5.1: symbolic phase plus the first numeric factorization on
// the CPU; its permutations and L/U structures are reused for every later
// system.)
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace kktlu {

struct AnalyzeOptions {
  int ordering = 0;       // 0 minimum degree on A+A^T, 1 natural, 2 user-supplied
  double tau = 1e-10;     // threshold partial pivoting
  int matching = 0;       // 1: maximum-product matching and scaling first (match_scale)
};

struct Analysis {
  int32_t n = 0;
  int64_t nnz = 0;
  std::vector<int32_t> Q, Qinv;  // Q[k] = original index of step k
  std::vector<int32_t> P, Pinv;  // P[k] = A'-row pivoted at step k
  // combined factors, CSR in pivot order: L strict part, diagonal, U strict part
  std::vector<int32_t> lu_rowptr;  // n+1
  std::vector<int32_t> lu_col;     // f
  std::vector<int32_t> diag;       // n, position of (i,i)
  std::vector<double> lu_val0;     // values from the pivoting pass
  std::vector<int32_t> lu_src;     // f, index into A's values or -1 (fill)
  // row dependency schedule (refactorization and L solve): rows by level
  std::vector<int32_t> lev_ptr, lev_rows;
  std::vector<int32_t> lev_maxlen;  // longest LU row of each level
  // U-solve schedule
  std::vector<int32_t> ulev_ptr, ulev_rows;
  // transposed views: column-major order of the strict L part and of U, as
  // positions into the CSR arrays (for the transposed solve)
  std::vector<int32_t> ut_ptr, ut_pos;   // column j of U: rows i<=j (diag last)
  std::vector<int32_t> lt_ptr, lt_pos;   // column j of strict L: rows i>j
  std::vector<int32_t> ltlev_ptr, ltlev_rows;  // L^T solve (descending) schedule
  std::vector<int32_t> utlev_ptr, utlev_rows;  // U^T solve (ascending) schedule
  int64_t nnz_l = 0, nnz_u = 0;
  int warn_singular = 0;
  // matching and scaling (empty without): the analysed matrix is
  // Ahat = Pm Dr A Dc, row j of Ahat being row match[j] of A scaled by
  // dr[match[j]] and column c by dc[c]; lu_src and the pivoting pass refer to
  // Ahat's values through A's positions; ascale[p] = dr[i] dc[j] for A's
  // stored entry p = (i, j) (powers of two: the scaled values are exact)
  std::vector<int32_t> match;
  std::vector<double> dr, dc, ascale;
};

// Maximum-product perfect matching of A's nonzero entries and power-of-two
// scaling from the canonical dual potentials (Section 5.2.1's MC64-style
// preprocessing): costs c_ij = log(cmax_j) - log|a_ij|, the minimum-cost
// perfect matching by successive shortest augmenting paths (Dijkstra over
// reduced costs with a binary heap), the largest column potentials v <= 0
// feasible with that matching (shortest distances from a source joined to
// every column, by a queue-based Bellman-Ford), u_i = c_{i,s(i)} - v_{s(i)},
// dr_i = 2^round(u_i / ln 2), dc_j = 2^round((v_j - log cmax_j) / ln 2).
// match[j] = row matched to column j.  Returns KKT_OK or
// KKT_ERR_STRUCTURALLY_SINGULAR (no perfect matching of nonzeros).
int match_scale(int32_t n, const int64_t* rowptr, const int32_t* colind, const double* val,
                std::vector<int32_t>& match, std::vector<double>& dr, std::vector<double>& dc);

// Status codes use the public enum's values.
int validate_csr(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colind,
                 std::string* msg);

// Exact minimum degree on pattern(A + A^T), ties -> smallest index.
void order_minimum_degree(int32_t n, const int64_t* rowptr, const int32_t* colind,
                          std::vector<int32_t>& Q);

// Full analysis.  Returns a kkt_status value; msg gets details on failure.
int analyze(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colind,
            const double* values0, const int32_t* user_q, const AnalyzeOptions& opt,
            Analysis& out, std::string* msg);

// The analysis of Ahat = Pm Dr A Dc for a given matching and scaling (used by
// analyze with opt.matching = 1 and by re-analysis, which keeps them): the
// result describes Ahat's factors with lu_src referring to A's positions and
// match, dr, dc, ascale set.
int analyze_scaled(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colind,
                   const double* values, const std::vector<int32_t>& match,
                   const std::vector<double>& dr, const std::vector<double>& dc,
                   const int32_t* user_q, const AnalyzeOptions& opt, Analysis& out,
                   std::string* msg);

// Batch of independent instances as one block-diagonal system: pattern p
// (n[p], nnz[p], rowptr[p], colind[p], values0[p]) is analysed once (patterns
// in parallel threads) and instance t is a copy of the analysis of pattern
// inst_pattern[t] with its rows and A positions offset; the level schedules
// are merged level by level.  row_off / nnz_off get the instance offsets
// (count + 1 entries).
int analyze_batch(int32_t npat, const int32_t* n, const int64_t* nnz,
                  const int64_t* const* rowptr, const int32_t* const* colind,
                  const double* const* values0, int32_t count, const int32_t* inst_pattern,
                  const AnalyzeOptions& opt, Analysis& out, std::vector<int64_t>& row_off,
                  std::vector<int64_t>& nnz_off, std::string* msg);

}  // namespace kktlu
