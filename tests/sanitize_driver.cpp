// Host-code sanitizer run (built by tests/test_sanitizers_cpu.py with
// -fsanitize=address,undefined): the host analysis of the library
// (analyze.cpp: ordering, pivoting pass, patterns, schedules, batch merge) and
// the oracle (factor, refactor, solve with refinement, transposed solve,
// gradient) on seeded random sparse matrices of many shapes, plus malformed
// CSR input that must be rejected.  Any out-of-bounds access, leak-free
// misuse or undefined behaviour aborts the run; the analysis and the oracle
// must also agree on the pivot sequence.  Prints "ok <cases>" on success.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

extern "C" {
#include "../oracle/oracle.h"
}
#include "../paper_2306_14337_amd/csrc/analyze.h"

namespace {

struct Csr {
  int32_t n = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
};

uint64_t g_state = 0x9E3779B97F4A7C15ull;
uint64_t next_u64() {
  g_state ^= g_state << 13;
  g_state ^= g_state >> 7;
  g_state ^= g_state << 17;
  return g_state;
}
double uniform() { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

// random pattern with a full diagonal (density d), values in [-1, 1] plus a
// diagonal shift (0 leaves pivoting real work to do)
Csr random_matrix(int32_t n, double d, double shift) {
  Csr a;
  a.n = n;
  a.rp.push_back(0);
  for (int32_t i = 0; i < n; i++) {
    for (int32_t j = 0; j < n; j++) {
      if (i == j || uniform() < d) {
        a.ci.push_back(j);
        a.v.push_back(2.0 * uniform() - 1.0 + (i == j ? shift : 0.0));
      }
    }
    a.rp.push_back((int64_t)a.ci.size());
  }
  return a;
}

int fail(const char* what, int n) {
  std::printf("FAIL %s (n=%d)\n", what, n);
  return 1;
}

}  // namespace

int main() {
  int cases = 0;
  const double taus[] = {1.0, 0.1, 1e-3, 1e-10};
  for (int32_t n : {1, 2, 3, 5, 8, 13, 21, 34, 60}) {
    for (double d : {0.05, 0.2, 0.6}) {
      for (double tau : taus) {
        const Csr a = random_matrix(n, d, tau < 1e-3 ? 4.0 : 0.0);
        kktlu::AnalyzeOptions opt;
        opt.tau = tau;
        kktlu::Analysis an;
        std::string msg;
        const int st = kktlu::analyze(a.n, (int64_t)a.ci.size(), a.rp.data(), a.ci.data(),
                                      a.v.data(), nullptr, opt, an, &msg);
        if (st < 0) return fail(msg.c_str(), n);
        int ost = 0;
        std::vector<int32_t> Qmd(n);
        if (oracle_order_md(a.n, a.rp.data(), a.ci.data(), Qmd.data()) != ORA_OK)
          return fail("oracle_order_md", n);
        oracle_lu* lu = oracle_factor(a.n, a.rp.data(), a.ci.data(), a.v.data(), Qmd.data(), tau, &ost);
        if (!lu) return fail("oracle_factor", n);
        // same pivot sequence (the independent codes follow one rule)
        std::vector<int32_t> P(n), Q(n);
        int64_t nl = 0, nu = 0;
        oracle_lu_sizes(lu, &nl, &nu);
        std::vector<int64_t> Lp(n + 1), Up(n + 1);
        std::vector<int32_t> Li(nl), Ui(nu);
        std::vector<double> Lx(nl), Ux(nu);
        oracle_lu_export(lu, P.data(), Q.data(), Lp.data(), Li.data(), Lx.data(), Up.data(),
                         Ui.data(), Ux.data());
        if (P != an.P || Q != an.Q) return fail("pivot sequence differs", n);
        // refactor, solves (both ops, two right-hand sides), gradient
        std::vector<double> v2 = a.v;
        for (double& x : v2) x *= 1.0 + 0.01 * (uniform() - 0.5);
        oracle_refactor(lu, v2.data(), 1e-18);
        std::vector<double> b(2 * (size_t)n), x(2 * (size_t)n), lam(2 * (size_t)n),
            g(a.ci.size());
        for (double& t : b) t = uniform() - 0.5;
        oracle_solve_opts so{};
        so.restart = 5;
        so.max_iters = 10;
        so.eta_target = 1e-12;
        oracle_solve_info si{};
        oracle_solve(lu, 'N', 2, b.data(), x.data(), &so, &si);
        oracle_solve(lu, 'T', 2, b.data(), lam.data(), &so, &si);
        oracle_grad(lu, 2, lam.data(), x.data(), g.data());
        oracle_lu_free(lu);
        cases++;
      }
    }
  }
  // block-diagonal batch of three patterns and five instances
  {
    std::vector<Csr> pats = {random_matrix(7, 0.3, 3.0), random_matrix(12, 0.2, 3.0),
                             random_matrix(4, 0.5, 3.0)};
    std::vector<int32_t> ns;
    std::vector<int64_t> nnzs;
    std::vector<const int64_t*> rps;
    std::vector<const int32_t*> cis;
    std::vector<const double*> vs;
    for (const Csr& p : pats) {
      ns.push_back(p.n);
      nnzs.push_back((int64_t)p.ci.size());
      rps.push_back(p.rp.data());
      cis.push_back(p.ci.data());
      vs.push_back(p.v.data());
    }
    const std::vector<int32_t> inst = {0, 1, 0, 2, 1};
    kktlu::AnalyzeOptions opt;
    kktlu::Analysis an;
    std::vector<int64_t> ro, no;
    std::string msg;
    const int st = kktlu::analyze_batch(3, ns.data(), nnzs.data(), rps.data(), cis.data(),
                                        vs.data(), (int32_t)inst.size(), inst.data(), opt, an, ro,
                                        no, &msg);
    if (st < 0) return fail(msg.c_str(), -1);
    cases++;
  }
  // malformed CSR: rejected, no access out of bounds
  {
    Csr a = random_matrix(6, 0.4, 2.0);
    std::string msg;
    std::vector<int32_t> bad = a.ci;
    bad[1] = 99;  // column out of range
    if (kktlu::validate_csr(a.n, (int64_t)bad.size(), a.rp.data(), bad.data(), &msg) >= 0)
      return fail("out-of-range column accepted", 6);
    std::vector<int64_t> rp = a.rp;
    rp[3] = rp[2] - 1;  // decreasing row pointer
    if (kktlu::validate_csr(a.n, (int64_t)a.ci.size(), rp.data(), a.ci.data(), &msg) >= 0)
      return fail("decreasing row pointers accepted", 6);
    cases++;
  }
  std::printf("ok %d\n", cases);
  return 0;
}
