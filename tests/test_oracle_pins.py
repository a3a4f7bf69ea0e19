"""Pins of the CPU oracle against facts fixed outside it: LAPACK getrf, brute
force with exactly rounded fma, the fill-path theorem, closed forms of the
minimum-degree ordering, textbook GMRES properties and the adjoint's closed
form.  CPU only.
"""
import itertools
import math
from fractions import Fraction
import os
from collections import deque

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from paper_2306_14337_amd import kktgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# independent helpers
# ---------------------------------------------------------------------------
def fma_exact(a, b, c):
    """Correctly rounded a*b + c (Fraction arithmetic, one rounding)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def dense_from_csr(n, rp, ci, v):
    D = np.zeros((n, n))
    M = np.zeros((n, n), dtype=bool)
    for i in range(n):
        D[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
        M[i, ci[rp[i]:rp[i + 1]]] = True
    return D, M


def csc_dense(n, p, i, x):
    D = np.zeros((n, n))
    M = np.zeros((n, n), dtype=bool)
    for j in range(n):
        D[i[p[j]:p[j + 1]], j] = x[p[j]:p[j + 1]]
        M[i[p[j]:p[j + 1]], j] = True
    return D, M


def brute_right_looking(Ad, Am, tau):
    """Dense right-looking elimination of A' with the threshold rule, tracking
    the structural pattern, exact fma.  Returns P, L, U (pivot order), masks."""
    n = Ad.shape[0]
    a = [[float(Ad[r, c]) for c in range(n)] for r in range(n)]
    S = [[bool(Am[r, c]) for c in range(n)] for r in range(n)]
    pivotal = [False] * n
    P = []
    Lcols = []  # (row, value) per step, rows are A'-rows
    Urows = []
    for k in range(n):
        cand = [r for r in range(n) if not pivotal[r] and S[r][k]]
        assert cand, "structurally singular"
        amax = max(abs(a[r][k]) for r in cand)
        has_d = k in cand
        if amax == 0.0:
            piv = k if has_d else min(cand)
        elif has_d and abs(a[k][k]) >= tau * amax and a[k][k] != 0.0:
            piv = k
        else:
            best = [r for r in cand if abs(a[r][k]) == amax]
            piv = min(best)
        pv = a[piv][k]
        P.append(piv)
        pivotal[piv] = True
        Urows.append({c: a[piv][c] for c in range(k, n) if S[piv][c]})
        col = []
        for r in cand:
            if r == piv:
                continue
            lval = a[r][k] / pv
            col.append((r, lval))
            for c in range(k + 1, n):
                if S[piv][c]:
                    if not S[r][c]:
                        S[r][c] = True
                        a[r][c] = 0.0
                    a[r][c] = fma_exact(-lval, a[piv][c], a[r][c])
        Lcols.append(col)
    step = {r: k for k, r in enumerate(P)}
    L = np.zeros((n, n))
    Lm = np.zeros((n, n), dtype=bool)
    U = np.zeros((n, n))
    Um = np.zeros((n, n), dtype=bool)
    for k in range(n):
        for r, v in Lcols[k]:
            L[step[r], k] = v
            Lm[step[r], k] = True
        for c, v in Urows[k].items():
            U[k, c] = v
            Um[k, c] = True
    return np.array(P), L, Lm, U, Um


def permuted(Ad, Am, Q):
    return Ad[np.ix_(Q, Q)], Am[np.ix_(Q, Q)]


# ---------------------------------------------------------------------------
# P1: dense LAPACK getrf (partial pivoting) agrees with tau = 1, Q = I
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed", [(1, 0), (5, 1), (17, 2), (64, 3)])
def test_dense_partial_pivoting_matches_lapack(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    rp = np.arange(0, n * n + 1, n, dtype=np.int64)
    ci = np.tile(np.arange(n, dtype=np.int32), n)
    lu = oracle.OracleLU(n, rp, ci, A.reshape(-1), Q=np.arange(n), tau=1.0)
    f = lu.factors()
    Pm, Ls, Us = sla.lu(A)
    P_lapack = np.argmax(Pm, axis=0)  # (Pm^T A)_i = A[P[i]]
    assert np.array_equal(f["P"], P_lapack)
    L, _ = csc_dense(n, f["Lp"], f["Li"], f["Lx"])
    U, _ = csc_dense(n, f["Up"], f["Ui"], f["Ux"])
    growth = np.abs(Us).max() / np.abs(A).max()
    assert np.allclose(L + np.eye(n), Ls, rtol=0, atol=1e-13 * max(growth, 1) * n)
    assert np.allclose(U, Us, rtol=0, atol=1e-13 * np.abs(Us).max() * n)


# ---------------------------------------------------------------------------
# Golden: hand-derived threshold LU (exact rationals)
# ---------------------------------------------------------------------------
def _read_golden(name):
    lines = [ln.split("#")[0].strip() for ln in open(os.path.join(GOLDEN, name))]
    lines = [ln for ln in lines if ln]
    n = int(lines[0].split()[1])
    A = np.array([[float(x) for x in lines[1 + i].split()] for i in range(n)])
    cases = []
    i = 1 + n
    while i < len(lines):
        tau = float(lines[i].split("=")[1])
        P = [int(x) for x in lines[i + 1].split()[1:]]

        def mat(s):
            return np.array([[float(Fraction(x)) for x in row.split()] for row in s.split(None, 1)[1].split("|")])

        cases.append((tau, P, mat(lines[i + 2]), mat(lines[i + 3])))
        i += 4
    return A, cases


def test_golden_threshold_lu_3x3():
    A, cases = _read_golden("threshold_lu_3x3.txt")
    n = A.shape[0]
    rp = np.arange(0, n * n + 1, n, dtype=np.int64)
    ci = np.tile(np.arange(n, dtype=np.int32), n)
    for tau, P, Lg, Ug in cases:
        lu = oracle.OracleLU(n, rp, ci, A.reshape(-1), Q=np.arange(n), tau=tau)
        f = lu.factors()
        assert list(f["P"]) == P
        L, _ = csc_dense(n, f["Lp"], f["Li"], f["Lx"])
        U, _ = csc_dense(n, f["Up"], f["Ui"], f["Ux"])
        assert np.allclose(L + np.eye(n), Lg, rtol=1e-15, atol=1e-15)
        assert np.allclose(U, Ug, rtol=1e-15, atol=1e-15)


# ---------------------------------------------------------------------------
# P2: brute-force right-looking elimination, bit for bit
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tau", [1.0, 0.1, 1e-3, 1e-10])
@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_pivots_pattern_values(tau, seed):
    n = 4 + seed * 2
    rp, ci, v = kktgen.random_sparse(n, 0.3, seed=100 + seed, diag=(seed % 2 == 0))
    # rows without any entry would be structurally singular; guarantee a transversal
    Ad, Am = dense_from_csr(n, rp, ci, v)
    if not all(Am.any(1)) or not all(Am.any(0)):
        Am = Am | np.eye(n, dtype=bool)
        Ad = Ad + np.eye(n) * (~dense_from_csr(n, rp, ci, v)[1] & np.eye(n, dtype=bool))
        r, c = np.nonzero(Am)
        rp = np.zeros(n + 1, np.int64)
        np.add.at(rp, r + 1, 1)
        rp = np.cumsum(rp)
        ci = c.astype(np.int32)
        v = Ad[r, c]
    Q = oracle.order_md(n, rp, ci)
    try:
        Pb, Lb, Lbm, Ub, Ubm = brute_right_looking(*permuted(Ad, Am, Q), tau)
    except AssertionError:
        with pytest.raises(ValueError):
            oracle.OracleLU(n, rp, ci, v, Q=Q, tau=tau)
        return
    lu = oracle.OracleLU(n, rp, ci, v, Q=Q, tau=tau)
    f = lu.factors()
    assert np.array_equal(f["P"], Pb)
    L, Lm = csc_dense(n, f["Lp"], f["Li"], f["Lx"])
    U, Um = csc_dense(n, f["Up"], f["Ui"], f["Ux"])
    assert np.array_equal(Lm, Lbm) and np.array_equal(Um, Ubm)
    assert np.array_equal(L, Lb) and np.array_equal(U, Ub)  # bitwise


@pytest.mark.parametrize("seed", range(3))
def test_bruteforce_tiny_kkt(seed):
    pat = kktgen.make_kkt(3 + seed, 500 + seed)
    vals = pat.values(kktgen.draw_sigma(np.random.default_rng(seed), pat.n_p))
    n = pat.n
    Ad, Am = dense_from_csr(n, pat.rowptr, pat.colind, vals)
    Q = oracle.order_md(n, pat.rowptr, pat.colind)
    for tau in (1.0, 1e-10):
        Pb, Lb, Lbm, Ub, Ubm = brute_right_looking(*permuted(Ad, Am, Q), tau)
        lu = oracle.OracleLU(n, pat.rowptr, pat.colind, vals, Q=Q, tau=tau)
        f = lu.factors()
        assert np.array_equal(f["P"], Pb)
        L, Lm = csc_dense(n, f["Lp"], f["Li"], f["Lx"])
        U, Um = csc_dense(n, f["Up"], f["Ui"], f["Ux"])
        assert np.array_equal(Lm, Lbm) and np.array_equal(Um, Ubm)
        assert np.array_equal(L, Lb) and np.array_equal(U, Ub)


def test_singular_column_continues():
    # second column has only zeros among the candidates -> warning, factor goes on
    A = np.array([[1.0, 0.0, 2.0], [3.0, 0.0, 1.0], [0.0, 0.0, 5.0]])
    M = np.array([[1, 1, 1], [1, 1, 1], [0, 0, 1]], dtype=bool)
    r, c = np.nonzero(M)
    rp = np.array([0, 3, 6, 7], np.int64)
    lu = oracle.OracleLU(3, rp, c.astype(np.int32), A[r, c], Q=np.arange(3), tau=1.0)
    assert lu.status == oracle.WARN_SINGULAR


def test_structurally_singular_rejected():
    # column 1 has no entry at all
    rp = np.array([0, 1, 2], np.int64)
    ci = np.array([0, 0], np.int32)
    with pytest.raises(ValueError):
        oracle.OracleLU(2, rp, ci, np.array([1.0, 2.0]), Q=np.arange(2), tau=1.0)


# ---------------------------------------------------------------------------
# P3: fill-path theorem (Rose-Tarjan) for the structural pattern of L+U
# ---------------------------------------------------------------------------
def fill_by_paths(M):
    """(i,j) in the filled pattern iff a path i -> j in G(M) uses only
    intermediate vertices numbered below min(i, j)."""
    n = M.shape[0]
    out = np.zeros_like(M)
    succ = [np.nonzero(M[i])[0] for i in range(n)]
    for i in range(n):
        for j in range(n):
            lim = min(i, j)
            seen = {i}
            dq = deque([i])
            found = False
            while dq and not found:
                u = dq.popleft()
                for w in succ[u]:
                    if w == j:
                        found = True
                        break
                    if w < lim and w not in seen:
                        seen.add(w)
                        dq.append(w)
            out[i, j] = found or (i == j and M[i, i])
    return out


@pytest.mark.parametrize("seed", range(4))
def test_fill_path_theorem(seed):
    n = 12 + 9 * seed
    rp, ci, v = kktgen.random_sparse(n, 0.12, seed=700 + seed, diag=True)
    v[rp[:-1]] += 0.0
    Ad, Am = dense_from_csr(n, rp, ci, v)
    Ad[np.diag_indices(n)] += 10.0 * np.sign(Ad[np.diag_indices(n)] + 1e-300) * n
    r, c = np.nonzero(Am)
    vals = Ad[r, c]
    Q = oracle.order_md(n, rp, ci)
    lu = oracle.OracleLU(n, rp, ci, vals, Q=Q, tau=0.5)
    f = lu.factors()
    Ap, Apm = permuted(Ad, Am, Q)
    PAm = Apm[f["P"], :]
    expect = fill_by_paths(PAm)
    _, Lm = csc_dense(n, f["Lp"], f["Li"], f["Lx"])
    _, Um = csc_dense(n, f["Up"], f["Ui"], f["Ux"])
    assert np.array_equal(Lm | Um, expect)


# ---------------------------------------------------------------------------
# P4: minimum-degree ordering
# ---------------------------------------------------------------------------
def graph_csr(n, edges):
    M = np.zeros((n, n), dtype=bool)
    for a, b in edges:
        M[a, b] = M[b, a] = True
    M |= np.eye(n, dtype=bool)
    r, c = np.nonzero(M)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, r + 1, 1)
    return np.cumsum(rp), c.astype(np.int32), M


def test_md_star_closed_form():
    n = 9
    rp, ci, _ = graph_csr(n, [(0, i) for i in range(1, n)])
    assert list(oracle.order_md(n, rp, ci)) == list(range(1, n - 1)) + [0, n - 1]


def test_md_path_closed_form():
    n = 11
    rp, ci, _ = graph_csr(n, [(i, i + 1) for i in range(n - 1)])
    assert list(oracle.order_md(n, rp, ci)) == list(range(n))


@pytest.mark.parametrize("n", [4, 7, 30])
def test_md_cycle_fill_closed_form(n):
    rp, ci, M = graph_csr(n, [(i, (i + 1) % n) for i in range(n)])
    Q = oracle.order_md(n, rp, ci)
    assert list(Q) == list(range(n))
    vals = np.where(np.eye(n, dtype=bool), 4.0, -1.0)[M]
    lu = oracle.OracleLU(n, rp, ci, vals, Q=Q, tau=1e-3)
    lnz, _ = lu.sizes()
    assert lnz == 2 * n - 3  # n cycle edges plus n-3 fill edges


@pytest.mark.parametrize("seed", range(5))
def test_md_tree_has_no_fill(seed):
    rng = np.random.default_rng(seed)
    n = 60
    edges = [(i, int(rng.integers(0, i))) for i in range(1, n)]
    rp, ci, M = graph_csr(n, edges)
    Q = oracle.order_md(n, rp, ci)
    vals = np.where(np.eye(n, dtype=bool), float(n), -1.0)[M]
    lu = oracle.OracleLU(n, rp, ci, vals, Q=Q, tau=1e-3)
    assert lu.sizes()[0] == n - 1


def md_by_reachable_sets(M):
    """Minimum degree where the degree of v is the number of uneliminated
    vertices reachable from v through eliminated ones (the elimination graph
    characterised by reachable sets; no explicit fill edges)."""
    n = M.shape[0]
    nb = [set(np.nonzero(M[i])[0]) - {i} for i in range(n)]
    elim = [False] * n
    order = []
    for _ in range(n):
        best = None
        for v in range(n):
            if elim[v]:
                continue
            seen = {v}
            stack = [v]
            deg = 0
            while stack:
                u = stack.pop()
                for w in nb[u]:
                    if w in seen:
                        continue
                    seen.add(w)
                    if elim[w]:
                        stack.append(w)
                    else:
                        deg += 1
            if best is None or deg < best[0]:
                best = (deg, v)
        order.append(best[1])
        elim[best[1]] = True
    return order


@pytest.mark.parametrize("seed", range(6))
def test_md_matches_reachable_set_definition(seed):
    n = 20 + 8 * seed
    rp, ci, v = kktgen.random_sparse(n, 2.5 / n, seed=900 + seed, diag=True, sym_pattern=seed % 2 == 0)
    _, Am = dense_from_csr(n, rp, ci, v)
    assert list(oracle.order_md(n, rp, ci)) == md_by_reachable_sets(Am | Am.T)


def test_md_kkt_small_matches_reachable_set_definition():
    pat = kktgen.make_kkt(5, 11)
    _, Am = dense_from_csr(pat.n, pat.rowptr, pat.colind, pat.base_values)
    assert list(oracle.order_md(pat.n, pat.rowptr, pat.colind)) == md_by_reachable_sets(Am)


# ---------------------------------------------------------------------------
# P5 / P6: refactorization
# ---------------------------------------------------------------------------
def test_refactor_of_first_matrix_is_bitwise_the_pivoting_pass():
    pat, seq = kktgen.make_sequence(100, 101, 1)
    v0 = seq[0][0]
    lu = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, v0, tau=1e-10)
    f0 = lu.factors()
    lu.refactor(v0)
    f1 = lu.factors()
    for k in ("Lx", "Ux"):
        assert np.array_equal(f0[k], f1[k])
    # backward error of the factorization
    n = pat.n
    Ad, _ = dense_from_csr(n, pat.rowptr, pat.colind, v0)
    Q, P = f0["Q"], f0["P"]
    PA = Ad[np.ix_(Q, Q)][P, :]
    L, _ = csc_dense(n, f0["Lp"], f0["Li"], f0["Lx"])
    U, _ = csc_dense(n, f0["Up"], f0["Ui"], f0["Ux"])
    err = np.abs(PA - (L + np.eye(n)) @ U).max()
    growth = np.abs(U).max() / np.abs(Ad).max()
    assert err <= 1e-13 * np.abs(Ad).sum(1).max() * max(growth, 1.0)


def doolittle_exact(PA, thr=0.0):
    """No-pivot dense LU, row by row, each entry updated in ascending k with a
    correctly rounded fma (the refactorization's arithmetic).  thr > 0: static
    pivoting, a finished pivot below thr in magnitude becomes copysign(thr)."""
    n = PA.shape[0]
    a = [[float(x) for x in row] for row in PA]
    for i in range(n):
        for k in range(i):
            l = a[i][k] / a[k][k]
            a[i][k] = l
            for j in range(k + 1, n):
                a[i][j] = fma_exact(-l, a[k][j], a[i][j])
        if thr > 0.0 and abs(a[i][i]) < thr:
            a[i][i] = math.copysign(thr, a[i][i])
    a = np.array(a)
    return np.tril(a, -1), np.triu(a)


@pytest.mark.parametrize("seed", range(3))
def test_refactor_matches_exact_doolittle(seed):
    pat = kktgen.make_kkt(3, 40 + seed)
    rng = np.random.default_rng(seed)
    v0 = pat.values(kktgen.draw_sigma(rng, pat.n_p))
    v1 = pat.values(kktgen.draw_sigma(rng, pat.n_p))
    lu = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, v0, tau=1e-10)
    lu.refactor(v1)
    f = lu.factors()
    n = pat.n
    Ad, _ = dense_from_csr(n, pat.rowptr, pat.colind, v1)
    PA = Ad[np.ix_(f["Q"], f["Q"])][f["P"], :]
    Ld, Ud = doolittle_exact(PA)
    L, Lm = csc_dense(n, f["Lp"], f["Li"], f["Lx"])
    U, Um = csc_dense(n, f["Up"], f["Ui"], f["Ux"])
    assert np.array_equal(L, Ld) and np.array_equal(U, Ud)
    # outside the structural pattern the dense factors are exactly zero
    assert not np.any(Ld[~Lm]) and not np.any(Ud[~Um])


@pytest.mark.parametrize("seed", range(3))
def test_refactor_static_pivoting_matches_exact_doolittle(seed):
    # threshold at the median pivot: about half of the pivots are raised
    pat = kktgen.make_kkt(3, 50 + seed)
    rng = np.random.default_rng(seed)
    v0 = pat.values(kktgen.draw_sigma(rng, pat.n_p))
    v1 = pat.values(kktgen.draw_sigma(rng, pat.n_p))
    lu = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, v0, tau=1e-10)
    lu.refactor(v1)
    piv = np.abs(lu.factors()["Ux"][np.diff(lu.factors()["Up"]).cumsum() - 1])
    anorm = np.abs(pat.scipy(v1)).sum(1).max()
    rel = float(np.median(piv)) / anorm
    assert lu.refactor(v1, perturb_rel=rel) == oracle.WARN_PERTURBED
    f = lu.factors()
    n = pat.n
    Ad, _ = dense_from_csr(n, pat.rowptr, pat.colind, v1)
    PA = Ad[np.ix_(f["Q"], f["Q"])][f["P"], :]
    Ld, Ud = doolittle_exact(PA, thr=rel * anorm)
    L, _ = csc_dense(n, f["Lp"], f["Li"], f["Lx"])
    U, _ = csc_dense(n, f["Up"], f["Ui"], f["Ux"])
    assert np.array_equal(L, Ld) and np.array_equal(U, Ud)
    assert np.abs(np.diag(U)).min() >= rel * anorm
    # threshold below every pivot: identical to the plain refactorization
    lu.refactor(v1)
    g = lu.factors()
    assert lu.refactor(v1, perturb_rel=0.5 * piv.min() / anorm) == oracle.OK
    assert np.array_equal(lu.factors()["Ux"], g["Ux"]) and np.array_equal(lu.factors()["Lx"], g["Lx"])


def test_refactor_tiny_pivot_warning():
    pat, seq = kktgen.make_sequence(100, 101, 1)
    lu = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, seq[0][0], tau=1e-10)
    assert lu.refactor(seq[0][0]) == oracle.OK
    assert lu.refactor(seq[0][0], tiny_rel=1e-6) == oracle.WARN_TINY_PIVOT


# ---------------------------------------------------------------------------
# P7: solves
# ---------------------------------------------------------------------------
def _eta(Ad, x, b):
    return np.abs(b - Ad @ x).max() / (np.abs(Ad).sum(1).max() * np.abs(x).max())


def test_solve_matches_dense_solve_well_conditioned():
    pat = kktgen.make_kkt(100, 101)
    rng = np.random.default_rng(5)
    sigma = np.clip(kktgen.draw_sigma(rng, pat.n_p), 1e-2, 1e2)
    vals = pat.values(sigma)
    vals[pat.rowptr[pat.n_p]:] = np.where(
        pat.colind[pat.rowptr[pat.n_p]:] >= pat.n_p, -1.0, vals[pat.rowptr[pat.n_p]:])
    b = rng.standard_normal(pat.n)
    Ad, _ = dense_from_csr(pat.n, pat.rowptr, pat.colind, vals)
    kappa = np.linalg.cond(Ad, 1)
    assert kappa < 1e10
    lu = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, vals, tau=1e-10)
    x, info = lu.solve(b)
    xd = np.linalg.solve(Ad, b)
    assert np.abs(x - xd).max() <= 1e-15 * kappa * np.abs(xd).max() * 10
    xt, info_t = lu.solve(b, op="T")
    assert np.abs(xt - np.linalg.solve(Ad.T, b)).max() <= 1e-15 * kappa * np.abs(xt).max() * 10


@pytest.mark.parametrize("B,seed", [(100, 101), (500, 7), (2000, 104)])
def test_eta_gate_on_kkt_sequences(B, seed):
    pat, seq = kktgen.make_sequence(B, seed, 3)
    lu = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, seq[0][0], tau=1e-10)
    A = None
    for vals, b in seq:
        lu.refactor(vals)
        x, info = lu.solve(b)
        A = pat.scipy(vals)
        eta = np.abs(b - A @ x).max() / (abs(A).sum(1).max() * np.abs(x).max())
        assert info["converged"] == 1 and eta <= 1e-12
        assert info["eta"] == pytest.approx(eta, rel=1e-6, abs=1e-30)


def test_transposed_solve_matches_dense():
    n = 30
    rp, ci, v = kktgen.random_sparse(n, 0.2, seed=31)
    Ad, _ = dense_from_csr(n, rp, ci, v)
    Ad += np.eye(n) * 0  # pattern unchanged
    lu = oracle.OracleLU(n, rp, ci, v, tau=1.0)
    b = np.random.default_rng(1).standard_normal((2, n))
    x = lu.apply(b[0], op="T")
    assert np.allclose(Ad.T @ x, b[0], atol=1e-10 * np.abs(b).max() * np.linalg.cond(Ad))
    x2, info = lu.solve(b.reshape(-1), op="T")
    for r in range(2):
        assert _eta(Ad.T, x2[r * n:(r + 1) * n], b[r]) <= 1e-12


# ---------------------------------------------------------------------------
# P8: FGMRES / CGS2 invariants
# ---------------------------------------------------------------------------
def test_arnoldi_relation_and_orthogonality():
    pat, seq = kktgen.make_sequence(100, 101, 2)
    lu = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, seq[0][0], tau=1e-10)
    lu.set_values(seq[1][0])  # stale preconditioner: a non-trivial Krylov space
    A = pat.scipy(seq[1][0])
    k, V, Z, H = lu.fgmres_trace(seq[1][1], 8, prec="L")
    assert k == 8
    Vk = V[:, :k + 1]
    lhs = A @ Z[:, :k]
    assert np.linalg.norm(lhs - Vk @ H[:k + 1, :k]) <= 1e-12 * abs(A).sum(1).max() * np.linalg.norm(Z[:, :k])
    assert np.abs(np.eye(k + 1) - Vk.T @ Vk).max() <= 1e-13


def test_gmres_identity_preconditioner_terminates_in_n_steps():
    n = 24
    rp, ci, v = kktgen.random_sparse(n, 0.3, seed=12)
    Ad, _ = dense_from_csr(n, rp, ci, v)
    Ad += 3 * np.eye(n) * np.sign(np.diag(Ad) + 1e-300)
    r, c = np.nonzero(dense_from_csr(n, rp, ci, v)[1])
    lu = oracle.OracleLU(n, rp, ci, Ad[r, c], tau=1.0)
    b = np.random.default_rng(2).standard_normal(n)
    k, V, Z, H = lu.fgmres_trace(b, n, prec="I")
    assert k <= n
    beta = np.linalg.norm(b)
    e1 = np.zeros(k + 1)
    e1[0] = beta
    y = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)[0]
    x = Z[:, :k] @ y
    assert np.linalg.norm(Ad @ x - b) <= 1e-9 * beta


def test_gmres_exact_preconditioner_one_step():
    n = 40
    rp, ci, v = kktgen.random_sparse(n, 0.2, seed=13)
    Ad, Am = dense_from_csr(n, rp, ci, v)
    Ad[np.diag_indices(n)] += 5.0
    r, c = np.nonzero(Am)
    lu = oracle.OracleLU(n, rp, ci, Ad[r, c], tau=1.0)
    b = np.random.default_rng(4).standard_normal(n)
    k, V, Z, H = lu.fgmres_trace(b, 3, prec="L")
    # A M^{-1} = I up to rounding: the Krylov space closes after one step and
    # the one-step least-squares iterate solves the system
    cond = np.linalg.cond(Ad)
    assert abs(H[1, 0]) <= 1e-14 * cond * abs(H[0, 0])
    x1 = Z[:, 0] * (np.linalg.norm(b) / H[0, 0])
    assert np.linalg.norm(Ad @ x1 - b) <= 1e-13 * cond * np.linalg.norm(b)


def test_fgmres_refines_stale_factor():
    pat = kktgen.make_kkt(500, 77)
    rng = np.random.default_rng(3)
    sigma = np.clip(kktgen.draw_sigma(rng, pat.n_p), 1e-2, 1e2)
    v_old = pat.values(sigma)
    v_new = v_old * (1.0 + 0.05 * rng.standard_normal(v_old.size))
    sym = pat.scipy(v_new)
    sym = (sym + sym.T) * 0.5
    sym.sort_indices()
    v_new = sym.data
    b = rng.standard_normal(pat.n)
    lu = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, v_old, tau=1e-10)
    lu.set_values(v_new)
    x, info = lu.solve(b)
    A = pat.scipy(v_new)
    eta = np.abs(b - A @ x).max() / (abs(A).sum(1).max() * np.abs(x).max())
    assert info["iters"] > 1 and info["converged"] == 1 and eta <= 1e-12
    # budget of zero iterations leaves the stale direct solve unconverged
    _, info0 = lu.solve(b, max_iters=0)
    assert info0["converged"] == 0 and info0["status"] == oracle.WARN_NOT_CONVERGED
    # min_iters forces refinement even when the direct solve is exact
    lu2 = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, v_old, tau=1e-10)
    _, info2 = lu2.solve(b, min_iters=2)
    assert info2["iters"] == 2 and info2["converged"] == 1


def test_iterative_refinement_steps_match_dense_definition():
    # classical refinement with a stale factor M = A1: x0 = A1^{-1} b and
    # x_{k+1} = x_k + A1^{-1} (b - A2 x_k), against dense numpy solves
    n = 60
    rp, ci, v = kktgen.random_sparse(n, 0.15, seed=21)
    A1, Am = dense_from_csr(n, rp, ci, v)
    A1[np.diag_indices(n)] += 6.0
    r, c = np.nonzero(Am)
    A2 = A1.copy()
    A2[r, c] *= 1.0 + 0.05 * np.random.default_rng(2).standard_normal(len(r))
    lu = oracle.OracleLU(n, rp, ci, A1[r, c], tau=1.0)
    lu.set_values(A2[r, c])
    b = np.random.default_rng(5).standard_normal(n)
    x = np.linalg.solve(A1, b)
    for k in range(1, 4):
        x = x + np.linalg.solve(A1, b - A2 @ x)
        xk, info = lu.solve(b, method="ir", max_iters=k, eta_target=0.0)
        assert info["iters"] == k
        assert np.abs(xk - x).max() <= 1e-12 * np.abs(x).max(), k
    # it converges linearly, at the rate of the stale factor's error
    rate = np.abs(np.linalg.eigvals(np.eye(n) - np.linalg.solve(A1, A2))).max()
    assert rate < 0.5
    xc, info = lu.solve(b, method="ir", max_iters=60)
    assert info["converged"] == 1
    assert np.abs(A2 @ xc - b).max() <= 1e-12 * np.abs(A2).sum(1).max() * np.abs(xc).max()
    # the same exit test and budget as FGMRES: zero iterations leave it stale
    _, info0 = lu.solve(b, method="ir", max_iters=0)
    assert info0["converged"] == 0 and info0["iters"] == 0


# ---------------------------------------------------------------------------
# P9: adjoint closed form dL/dA = -A^{-T} C X^T on the pattern
# ---------------------------------------------------------------------------
def test_gradient_closed_form():
    n, nrhs = 40, 3
    rp, ci, v = kktgen.random_sparse(n, 0.15, seed=55)
    Ad, Am = dense_from_csr(n, rp, ci, v)
    Ad[np.diag_indices(n)] += 4.0
    r, c = np.nonzero(Am)
    vals = Ad[r, c]
    lu = oracle.OracleLU(n, rp, ci, vals, tau=1.0)
    rng = np.random.default_rng(8)
    Bm = rng.standard_normal((nrhs, n))
    Cm = rng.standard_normal((nrhs, n))
    x, _ = lu.solve(Bm.reshape(-1))
    lam, _ = lu.solve(Cm.reshape(-1), op="T")
    g = lu.grad(lam, x)
    Ainv = np.linalg.inv(Ad)
    X = Ainv @ Bm.T
    G = -(Ainv.T @ Cm.T) @ X.T
    assert np.allclose(g, G[r, c], rtol=1e-9, atol=1e-11 * np.abs(G).max())
    # finite differences of L = sum_r c_r^T x_r on a few entries
    h = 1e-6
    for p in range(0, len(vals), max(1, len(vals) // 7)):
        dA = np.zeros_like(Ad)
        dA[r[p], c[p]] = h
        Lp = np.sum(Cm.T * np.linalg.solve(Ad + dA, Bm.T))
        Lm_ = np.sum(Cm.T * np.linalg.solve(Ad - dA, Bm.T))
        assert (Lp - Lm_) / (2 * h) == pytest.approx(g[p], rel=1e-5, abs=1e-7)


# ---------------------------------------------------------------------------
# |L||U|, growth figure and sweep-based triangular solves
# ---------------------------------------------------------------------------
def _dense_factors(ora):
    f = ora.factors()
    n = ora.n
    L, _ = csc_dense(n, f["Lp"], f["Li"], f["Lx"])
    U, Um = csc_dense(n, f["Up"], f["Ui"], f["Ux"])
    return f, L + np.eye(n), U, Um


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_absprod_matches_dense_product(seed):
    # (|L||U|)_ij on the pattern equals the dense product of the absolute
    # factors (unit diagonal of L included), for L and U entries alike
    n = 30 + 5 * seed
    rp, ci, v = kktgen.random_sparse(n, 0.12, seed=400 + seed)
    ora = oracle.OracleLU(n, rp, ci, v, tau=0.1)
    f, L, U, _ = _dense_factors(ora)
    ref = np.abs(L) @ np.abs(U)
    sL, sU = ora.absprod()
    for j in range(n):
        for t in range(f["Up"][j], f["Up"][j + 1]):
            i = f["Ui"][t]
            assert abs(sU[t] - ref[i, j]) <= 1e-13 * ref[i, j], (i, j)
        for t in range(f["Lp"][j], f["Lp"][j + 1]):
            i = f["Li"][t]
            assert abs(sL[t] - ref[i, j]) <= 1e-13 * ref[i, j], (i, j)


@pytest.mark.parametrize("n", [2, 5, 12, 30])
def test_growth_wilkinson_closed_form(n):
    # Wilkinson's matrix (1 on the diagonal, -1 below it, 1 in the last
    # column) under partial pivoting keeps the diagonal pivots and doubles the
    # last column at every step: max |U| = u_nn = 2^(n-1) and ||A||_inf = n
    A = np.eye(n) - np.tril(np.ones((n, n)), -1)
    A[:, -1] = 1.0
    rp, ci, v = [0], [], []
    for i in range(n):
        for j in range(n):
            if A[i, j] != 0.0:
                ci.append(j)
                v.append(A[i, j])
        rp.append(len(ci))
    ora = oracle.OracleLU(n, np.array(rp), np.array(ci), np.array(v),
                          Q=np.arange(n, dtype=np.int32), tau=1.0)
    assert np.array_equal(ora.factors()["P"], np.arange(n))
    assert ora.growth() == 2.0 ** (n - 1) / n


def test_growth_tracks_refactorization():
    # after a refactorization the figure is that of the new factors: scaling
    # the matrix leaves it unchanged, and a matrix whose U is known (upper
    # triangular A with Q = P = identity) gives max|a_ij| / ||A||_inf
    n = 40
    rp, ci, v = kktgen.random_sparse(n, 0.1, seed=77)
    ora = oracle.OracleLU(n, rp, ci, v, tau=1e-10)
    g0 = ora.growth()
    ora.refactor(v * 1024.0)
    assert ora.growth() == g0
    D = np.triu(np.random.default_rng(5).normal(size=(n, n))) + 5 * np.eye(n)
    rp2 = np.concatenate([[0], np.cumsum(np.arange(n, 0, -1))]).astype(np.int64)
    ci2 = np.concatenate([np.arange(i, n) for i in range(n)]).astype(np.int32)
    v2 = np.concatenate([D[i, i:] for i in range(n)])
    o2 = oracle.OracleLU(n, rp2, ci2, v2, Q=np.arange(n, dtype=np.int32), tau=1e-10)
    ref = np.abs(D).max() / np.abs(D).sum(1).max()
    assert abs(o2.growth() - ref) <= 1e-15 * ref  # row sums rounded in another order


def _jacobi_setup(seed):
    n = 36
    rp, ci, v = kktgen.random_sparse(n, 0.1, seed=500 + seed)
    ora = oracle.OracleLU(n, rp, ci, v, tau=0.1)
    f, L, U, _ = _dense_factors(ora)
    pin = f["Q"][f["P"]]
    return n, ora, f, L, U, pin


@pytest.mark.parametrize("seed", [0, 1])
def test_jacobi_sweeps_partial_neumann_sums(seed):
    # k sweeps from the right-hand side unroll into partial Neumann sums:
    # y_k = sum_{j<=k} (-L_s)^j c and, with U = D (I + N), N = D^{-1} U_s and
    # z_0 = y_k, z_k = sum_{j<k} (-N)^j D^{-1} y_k + (-N)^k y_k
    n, ora, f, L, U, pin = _jacobi_setup(seed)
    b = np.random.default_rng(seed).normal(size=n)
    c = b[pin]
    Ls = L - np.eye(n)
    d = np.diag(U)
    N = (U - np.diag(d)) / d[:, None]
    for k in (0, 1, 2, 5):
        y = sum(np.linalg.matrix_power(-Ls, j) @ c for j in range(k + 1))
        z = np.linalg.matrix_power(-N, k) @ y
        for j in range(k):
            z = z + np.linalg.matrix_power(-N, j) @ (y / d)
        x = np.empty(n)
        x[f["Q"]] = z
        xo = ora.apply_jacobi(b, k)
        assert np.abs(xo - x).max() <= 1e-10 * np.abs(x).max(), k


def test_jacobi_one_sweep_closed_form():
    # one sweep: z = D^{-1} (I - U_s) (I - L_s) c
    n, ora, f, L, U, pin = _jacobi_setup(3)
    b = np.random.default_rng(9).normal(size=n)
    d = np.diag(U)
    z = ((np.eye(n) - (U - np.diag(d))) @ ((2 * np.eye(n) - L) @ b[pin])) / d
    x = np.empty(n)
    x[f["Q"]] = z
    assert np.abs(ora.apply_jacobi(b, 1) - x).max() <= 1e-12 * np.abs(x).max()


def test_jacobi_depth_sweeps_exact():
    # as many sweeps as the longer triangle's dependency depth reproduce the
    # exact triangular solves (scipy's dense triangular solver)
    n, ora, f, L, U, pin = _jacobi_setup(4)
    b = np.random.default_rng(11).normal(size=n)
    y = sla.solve_triangular(L, b[pin], lower=True, unit_diagonal=True)
    z = sla.solve_triangular(U, y, lower=False)
    x = np.empty(n)
    x[f["Q"]] = z
    xo = ora.apply_jacobi(b, n)
    assert np.abs(xo - x).max() <= 1e-10 * np.abs(x).max()
    # fewer sweeps than the depth differ (the test has teeth)
    depth = 0
    Lm = np.abs(L - np.eye(n)) > 0
    lev = np.zeros(n, int)
    for i in range(n):
        js = np.nonzero(Lm[i, :i])[0]
        lev[i] = 1 + lev[js].max() if js.size else 0
    depth = lev.max()
    if depth >= 2:
        assert np.abs(ora.apply_jacobi(b, depth - 1) - x).max() > 1e-8 * np.abs(x).max()


# ---------------------------------------------------------------------------
# Maximum-product matching and power-of-two scaling (Section 5.2.1)
# ---------------------------------------------------------------------------
def _perm_product_argmax(A):
    n = A.shape[0]
    best, arg = -1.0, None
    for perm in itertools.permutations(range(n)):
        # perm[i] = column of row i
        p = 1.0
        for i in range(n):
            p *= abs(A[i, perm[i]])
        if p > best:
            best, arg = p, perm
    return best, arg


@pytest.mark.parametrize("n,density,seed", [(3, 0.5, 1), (5, 0.4, 2), (6, 0.3, 3), (7, 0.35, 4),
                                            (7, 0.8, 5), (6, 0.6, 6)])
def test_matching_is_brute_force_max_product(n, density, seed):
    rp, ci, v = kktgen.random_sparse(n, density, seed=seed)
    A = sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()
    best, arg = _perm_product_argmax(A)
    match, dr, dc = oracle.match_scale(n, rp, ci, v)
    col_of_row = np.empty(n, dtype=np.int64)
    col_of_row[match] = np.arange(n)
    assert tuple(col_of_row) == tuple(arg)
    got = np.prod(np.abs(A[np.arange(n), col_of_row]))
    assert got == best


@pytest.mark.parametrize("seed", range(4))
def test_scaling_bounds(seed):
    n = 40
    rp, ci, v = kktgen.random_sparse(n, 0.15, seed=100 + seed)
    v = v * 10.0 ** np.random.default_rng(seed).uniform(-6, 6, v.size)
    match, dr, dc = oracle.match_scale(n, rp, ci, v)
    A = sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()
    S = dr[:, None] * A * dc[None, :]
    assert np.abs(S).max() <= 2.0
    d = np.abs(S[match, np.arange(n)])
    assert d.min() >= 0.5 and d.max() <= 2.0
    # powers of two only: the scaled values are exact
    assert np.all(np.frexp(dr)[0] == 0.5) and np.all(np.frexp(dc)[0] == 0.5)


def test_matching_permuted_diagonal_closed_form():
    # a permuted diagonal matrix with power-of-two magnitudes: the matching is
    # the permutation and the scaled matched entries are exactly +-1
    n = 9
    rng = np.random.default_rng(7)
    perm = rng.permutation(n)
    vals = (2.0 ** rng.integers(-20, 20, n)) * rng.choice([-1.0, 1.0], n)
    A = np.zeros((n, n))
    A[np.arange(n), perm] = vals
    Acsr = sp.csr_matrix(A)
    match, dr, dc = oracle.match_scale(n, Acsr.indptr, Acsr.indices, Acsr.data)
    assert np.array_equal(match[perm], np.arange(n))
    S = dr[:, None] * A * dc[None, :]
    assert np.array_equal(np.abs(S[np.arange(n), perm]), np.ones(n))


def test_matching_reports_structural_singularity():
    # row 2 is all zero values: no perfect matching of nonzeros
    rp = np.array([0, 2, 5, 6])
    ci = np.array([0, 1, 0, 1, 2, 1], dtype=np.int32)
    v = np.array([1.0, 2.0, 0.5, 1.0, 3.0, 0.0])
    with pytest.raises(ValueError):
        oracle.match_scale(3, rp, ci, v)


def test_matched_scaled_matrix_of_a_kkt_system():
    # the KKT (2,2) block is -1e-8 I: the matching prefers the O(1) entries
    # of J, and the matched, scaled matrix has entries of at most 2
    pat, seq = kktgen.make_sequence(10, 3, 1)
    vals = seq[0][0]
    match, dr, dc = oracle.match_scale(pat.n, pat.rowptr, pat.colind, vals)
    assert np.array_equal(np.sort(match), np.arange(pat.n))
    rp, ci, sv, src = oracle.matched_scaled(pat.n, pat.rowptr, pat.colind, vals, match, dr, dc)
    S = sp.csr_matrix((sv, ci, rp), shape=(pat.n, pat.n))
    assert abs(S).max() <= 2.0
    assert np.all(np.abs(S.diagonal()) >= 0.5)
    A = pat.scipy(vals)
    # the row permutation and scaling are exact: S = diag(dr)[match] A diag(dc)
    ref = (sp.diags(dr) @ A @ sp.diags(dc)).tocsr()[match]
    assert np.array_equal(S.toarray(), ref.toarray())
