"""GPU path vs the CPU oracle, through the C ABI (needs an MI355X).

* refactorization: the factor values equal the oracle's refactorization bit
  for bit (both apply each entry's updates in ascending pivot order with fma),
  which implies the headline metric ||F_gpu - F_ora||_F / ||F_ora||_F <= 1e-10;
* solve: backward error eta = ||b - A x||_inf / (||A||_inf ||x||_inf) <= 1e-12
  after refinement, for op 'N' and 'T';
* refinement: forced iterations and stale factors converge; a zero budget
  reports non-convergence;
* adjoint: gradient on the pattern vs the oracle's;
* edge cases: ragged tiny systems, several right-hand sides, error statuses.
"""
import numpy as np
import scipy.sparse as sp
import pytest

import oracle
from paper_2306_14337_amd import binding, kktgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def oracle_csr_values(lu: oracle.OracleLU):
    f = lu.factors()
    n = lu.n
    rows = np.concatenate([f["Li"], f["Ui"]])
    cols = np.concatenate([np.repeat(np.arange(n), np.diff(f["Lp"])),
                           np.repeat(np.arange(n), np.diff(f["Up"]))])
    vals = np.concatenate([f["Lx"], f["Ux"]])
    return vals[np.lexsort((cols, rows))]


def eta(A, x, b):
    return np.abs(b - A @ x).max() / (abs(A).sum(1).max() * np.abs(x).max())


def assert_factors_equal(gpu_vals, ora_vals):
    print(f"  factor entries {len(ora_vals)}", flush=True)
    rel = np.linalg.norm(gpu_vals - ora_vals) / np.linalg.norm(ora_vals)
    assert rel <= 1e-10, rel
    assert np.array_equal(gpu_vals.view(np.int64), ora_vals.view(np.int64)), (
        f"not bitwise equal ({np.sum(gpu_vals != ora_vals)} entries differ, rel {rel:.3e})")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()
    yield


# (schedule, sync_mode): level-synchronous launches; dependency-driven with
# acquire/release fences; dependency-driven with device-coherent accesses
SCHEDULES = [(1, 0), (2, 1), (2, 2)]


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("B,seed,steps", [(3, 5, 2), (100, 101, 3), (500, 7, 3), (2000, 104, 3)])
def test_sequence_refactor_solve(B, seed, steps, schedule):
    print(f"case B={B} seed={seed} schedule={schedule}", flush=True)
    pat, seq = kktgen.make_sequence(B, seed, steps)
    s = binding.KKTSolver(schedule=schedule[0], sync_mode=schedule[1])
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, seq[0][0], tau=1e-10)
    # before any refactorization the handle holds the pivoting pass's factors
    assert_factors_equal(s.lu()[2], oracle_csr_values(ora))
    for k, (vals, b) in enumerate(seq):
        s.refactor(dev(vals))
        x = s.solve(dev(b))
        rep = s.report()
        ora.refactor(vals)
        assert_factors_equal(s.lu()[2], oracle_csr_values(ora))
        A = pat.scipy(vals)
        xh = x.cpu().numpy()
        e = eta(A, xh, b)
        print(f"  step {k}: eta {e:.3e} iters {rep.iters}", flush=True)
        assert e <= 1e-12
        # the device's own eta agrees up to the rounding of the residual itself
        # (both are far below 1e-12 here; summation orders differ)
        assert rep.eta <= 1e-12 and abs(rep.eta - e) <= 1e-15
        xo, info = ora.solve(b)
        assert info["converged"] == 1


@pytest.mark.parametrize("variant", [dict(refactor_map=-1), dict(refactor_short_rows=-1),
                                     dict(refactor_long_rows=-1),
                                     dict(refactor_short_rows=-1, refactor_long_rows=-1),
                                     dict(refactor_micro_rows=-1)],
                         ids=["binary-search", "short-rows-pivot-by-pivot", "long-rows-wave-per-row",
                              "wave-per-row-everywhere", "no-micro-rows"])
@pytest.mark.parametrize("B,seed", [(100, 101), (2000, 104)])
def test_refactor_kernel_variants_bitwise(B, seed, variant):
    # binary search of each update's column instead of the precomputed map;
    # the short-row band pivot by pivot instead of as one list of updates;
    # one wave per long row instead of a workgroup; a wave for every short row
    # (no micro rows taken one per lane)
    print(f"case B={B} seed={seed} {variant}", flush=True)
    pat, seq = kktgen.make_sequence(B, seed, 2)
    s = binding.KKTSolver(schedule=2, sync_mode=2, **variant)
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, seq[0][0], tau=1e-10)
    for vals, b in seq:
        s.refactor(dev(vals))
        ora.refactor(vals)
        assert_factors_equal(s.lu()[2], oracle_csr_values(ora))


@pytest.mark.parametrize("B,seed,tail", [
    (3, 5, 26),       # the whole matrix is the dense block (n = 26, padded to 32)
    (100, 101, 100),  # padded block, ragged last panel
    (500, 7, 256),
    (10000, 102, 0),  # automatic size (384 at this size)
    (2000, 104, 700),
    (10000, 102, 2048),  # the largest dense block: 64 panels, 64 block solves
])
@pytest.mark.parametrize("dense_lu", [0, 1], ids=["panel-launches", "task-launch"])
def test_dense_tail_bitwise(B, seed, tail, dense_lu):
    # the trailing block finished as a dense LU gives the oracle's factors bit
    # for bit (same update order), before and after a change of values, with
    # a panel and an update launch per 32 pivots or one task launch
    print(f"case B={B} seed={seed} dense_tail={tail} dense_lu={dense_lu}", flush=True)
    pat, seq = kktgen.make_sequence(B, seed, 2)
    s = binding.KKTSolver(schedule=2, sync_mode=2, dense_tail=tail, dense_lu=dense_lu)
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    got = s.info().dense_tail
    print(f"  dense tail {got}", flush=True)
    if tail > 0:
        assert got == min(tail, pat.n)
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, seq[0][0], tau=1e-10)
    for vals, b in seq:
        s.refactor(dev(vals))
        ora.refactor(vals)
        assert_factors_equal(s.lu()[2], oracle_csr_values(ora))
        x = s.solve(dev(b)).cpu().numpy()
        assert eta(pat.scipy(vals), x, b) <= 1e-12
        xt = s.solve(dev(b), op="T").cpu().numpy()
        assert eta(pat.scipy(vals).T.tocsr(), xt, b) <= 1e-12


# solve layouts: chain blocks (solve_chain) with and without the dense block;
# the older level-chunk + one-workgroup segment path (solve_chain=-1) for
# several segment widths
SOLVE_LAYOUTS = [
    dict(solve_chain=0), dict(solve_chain=1), dict(solve_chain=8),
    dict(solve_chain=0, dense_tail=-1), dict(solve_chain=0, dense_tail=200),
    dict(solve_chain=-1, solve_thin_rows=-1), dict(solve_chain=-1, solve_thin_rows=1),
    dict(solve_chain=-1, solve_thin_rows=16), dict(solve_chain=-1, solve_thin_rows=40),
    dict(solve_chain=-1, solve_thin_rows=256),
]


@pytest.mark.parametrize("layout", SOLVE_LAYOUTS, ids=lambda d: "-".join(f"{k}{v}" for k, v in d.items()))
@pytest.mark.parametrize("B,seed", [(3, 5), (500, 7), (2000, 104)])
def test_direct_solve_matches_oracle_apply(B, seed, layout):
    # no refinement: the GPU's x = Q U^-1 L^-1 P Q^T b (and the transposed
    # chain) against the oracle's
    print(f"case B={B} seed={seed} {layout}", flush=True)
    pat, seq = kktgen.make_sequence(B, seed, 1)
    vals, b = seq[0]
    opts = dict(layout)
    if opts.get("dense_tail", 0) > pat.n:
        opts["dense_tail"] = pat.n
    s = binding.KKTSolver(schedule=2, sync_mode=2, fgmres_max_iters=0, **opts)
    s.analyze(pat.n, pat.rowptr, pat.colind, vals)
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, vals, tau=1e-10)
    A = pat.scipy(vals)
    # first with the analysis's own factors, then after a refactorization
    for stage in ("analysis", "refactor"):
        if stage == "refactor":
            s.refactor(dev(vals))
        for op, M in (("N", A), ("T", A.T.tocsr())):
            x = s.solve(dev(b), op=op).cpu().numpy()
            xo = ora.apply(b, op)
            # the two differ only in the summation order inside each row
            err = np.abs(x - xo).max() / np.abs(xo).max()
            print(f"  {stage} op {op}: rel diff {err:.3e} eta {eta(M, x, b):.3e} "
                  f"oracle eta {eta(M, xo, b):.3e}", flush=True)
            assert err <= 1e-8, (stage, op, err)
            assert eta(M, x, b) <= max(100 * eta(M, xo, b), 1e-14), (stage, op)


@pytest.mark.parametrize("layout", [dict(), dict(dense_tail=300), dict(dense_tail=-1),
                                    dict(solve_chain=-1)],
                         ids=lambda d: "-".join(f"{k}{v}" for k, v in d.items()) or "default")
def test_direct_multi_rhs_matches_oracle_apply(layout):
    # eleven columns: one pass of eight and one of three (both kernel widths),
    # no refinement, each column against the oracle's direct solve
    pat, seq = kktgen.make_sequence(2000, 104, 1)
    vals, _ = seq[0]
    s = binding.KKTSolver(schedule=2, sync_mode=2, fgmres_max_iters=0, **layout)
    s.analyze(pat.n, pat.rowptr, pat.colind, vals)
    s.refactor(dev(vals))
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, vals, tau=1e-10)
    B = np.random.default_rng(11).standard_normal((11, pat.n))
    for op in ("N", "T"):
        X = s.solve(dev(B.reshape(-1)), op=op).cpu().numpy().reshape(11, pat.n)
        for r in range(11):
            xo = ora.apply(B[r], op)
            err = np.abs(X[r] - xo).max() / np.abs(xo).max()
            assert err <= 1e-8, (layout, op, r, err)


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_transposed_solve_and_multiple_rhs(schedule):
    pat, seq = kktgen.make_sequence(500, 9, 1)
    vals, _ = seq[0]
    s = binding.KKTSolver(schedule=schedule[0], sync_mode=schedule[1])
    s.analyze(pat.n, pat.rowptr, pat.colind, vals)
    s.refactor(dev(vals))
    rng = np.random.default_rng(3)
    B = rng.standard_normal((4, pat.n))
    A = pat.scipy(vals)
    for op, M in (("N", A), ("T", A.T.tocsr())):
        X = s.solve(dev(B.reshape(-1)), op=op).cpu().numpy().reshape(4, pat.n)
        for r in range(4):
            assert eta(M, X[r], B[r]) <= 1e-12, (op, r)


@pytest.mark.parametrize("refine_sync", [0, 1], ids=["device-checked", "host-checked"])
def test_refinement_forced_and_stale(refine_sync):
    pat = kktgen.make_kkt(500, 77)
    rng = np.random.default_rng(3)
    sigma = np.clip(kktgen.draw_sigma(rng, pat.n_p), 1e-2, 1e2)
    v_old = pat.values(sigma)
    sym = pat.scipy(v_old * (1.0 + 0.05 * rng.standard_normal(v_old.size)))
    sym = (sym + sym.T) * 0.5
    sym.sort_indices()
    v_new = sym.data
    b = rng.standard_normal(pat.n)
    A_new = pat.scipy(v_new)
    # forced iterations on an exact factorization
    s = binding.KKTSolver(min_iters=2, refine_sync=refine_sync)
    s.analyze(pat.n, pat.rowptr, pat.colind, v_old)
    s.refactor(dev(v_old))
    x = s.solve(dev(b)).cpu().numpy()
    assert s.report().iters == 2 and eta(pat.scipy(v_old), x, b) <= 1e-12
    # stale factors: FGMRES makes up the difference
    s = binding.KKTSolver(refine_sync=refine_sync)
    s.analyze(pat.n, pat.rowptr, pat.colind, v_old)
    s.refactor(dev(v_old))
    s.update_matrix(dev(v_new))
    x = s.solve(dev(b)).cpu().numpy()
    rep = s.report()
    print(f"  stale: iters {rep.iters} eta {rep.eta:.3e}", flush=True)
    assert rep.iters > 1 and eta(A_new, x, b) <= 1e-12
    # a restart inside the budget (restart length 4): same target
    s4 = binding.KKTSolver(refine_sync=refine_sync, fgmres_restart=4)
    s4.analyze(pat.n, pat.rowptr, pat.colind, v_old)
    s4.refactor(dev(v_old))
    s4.update_matrix(dev(v_new))
    x4 = s4.solve(dev(b)).cpu().numpy()
    rep4 = s4.report()
    print(f"  stale, restart 4: iters {rep4.iters} eta {rep4.eta:.3e}", flush=True)
    assert rep4.iters > 4 and eta(A_new, x4, b) <= 1e-12
    # zero budget: warning, not an error (reported by the solve itself only
    # when the host checks eta; always by the report)
    s0 = binding.KKTSolver(fgmres_max_iters=0, refine_sync=refine_sync)
    s0.analyze(pat.n, pat.rowptr, pat.colind, v_old)
    s0.refactor(dev(v_old))
    s0.update_matrix(dev(v_new))
    s0.solve(dev(b))
    if refine_sync:
        assert s0.last_status == binding.WARN_NOT_CONVERGED
    assert s0.report().warnings & (1 << binding.WARN_NOT_CONVERGED)
    # a launch budget below the iterations needed: the same warning
    s1 = binding.KKTSolver(refine_budget=1)
    s1.analyze(pat.n, pat.rowptr, pat.colind, v_old)
    s1.refactor(dev(v_old))
    s1.update_matrix(dev(v_new))
    s1.solve(dev(b))
    rep1 = s1.report()
    assert rep1.iters == 1 and rep1.warnings & (1 << binding.WARN_NOT_CONVERGED)


@pytest.mark.parametrize("refine_sync", [0, 1], ids=["device-checked", "host-checked"])
@pytest.mark.parametrize("op", ["N", "T"])
def test_classical_refinement_matches_oracle(op, refine_sync):
    # refine=1 with stale factors: same method as the oracle's "ir"; the
    # iterates differ only by rounding, so the iteration counts agree to one
    pat = kktgen.make_kkt(500, 78)
    rng = np.random.default_rng(4)
    sigma = np.clip(kktgen.draw_sigma(rng, pat.n_p), 1e-2, 1e2)
    v_old = pat.values(sigma)
    sym = pat.scipy(v_old * (1.0 + 0.005 * rng.standard_normal(v_old.size)))
    sym = (sym + sym.T) * 0.5
    sym.sort_indices()
    v_new = sym.data
    b = rng.standard_normal(pat.n)
    s = binding.KKTSolver(refine=1, fgmres_max_iters=40, refine_sync=refine_sync)
    s.analyze(pat.n, pat.rowptr, pat.colind, v_old)
    s.refactor(dev(v_old))
    s.update_matrix(dev(v_new))
    x = s.solve(dev(b), op=op).cpu().numpy()
    rep = s.report()
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, v_old, tau=1e-10)
    ora.set_values(v_new)
    xo, info = ora.solve(b, op=op, method="ir", max_iters=40)
    M = pat.scipy(v_new) if op == "N" else pat.scipy(v_new).T.tocsr()
    print(f"  op {op}: gpu iters {rep.iters} eta {rep.eta:.3e}; oracle iters {info['iters']}",
          flush=True)
    assert info["converged"] == 1 and rep.iters > 1
    assert eta(M, x, b) <= 1e-12
    assert abs(rep.iters - info["iters"]) <= 1
    assert np.abs(x - xo).max() <= 1e-6 * np.abs(xo).max()


@pytest.mark.parametrize("layout", [dict(schedule=2, sync_mode=2), dict(schedule=2, sync_mode=2, dense_tail=300),
                                    dict(schedule=2, sync_mode=2, dense_tail=300, dense_lu=1),
                                    dict(schedule=1), dict(schedule=2, sync_mode=1)],
                         ids=["coherent", "dense-block", "dense-block-tasks", "levels", "fences"])
def test_static_pivoting_bitwise(layout):
    # threshold at the median pivot magnitude: about half of the pivots are
    # raised, identically in every refactorization kernel and in the oracle
    pat, seq = kktgen.make_sequence(500, 7, 2)
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, seq[0][0], tau=1e-10)
    vals = seq[1][0]
    ora.refactor(vals)
    f = ora.factors()
    piv = np.abs(f["Ux"][np.diff(f["Up"]).cumsum() - 1])
    anorm = np.abs(pat.scipy(vals)).sum(1).max()
    rel = float(np.median(piv)) / anorm
    assert ora.refactor(vals, perturb_rel=rel) == oracle.WARN_PERTURBED
    s = binding.KKTSolver(pivot_perturb_rel=rel, **layout)
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    s.refactor(dev(vals))
    assert_factors_equal(s.lu()[2], oracle_csr_values(ora))
    assert s.report().warnings & (1 << binding.WARN_PERTURBED_PIVOT)
    # a threshold that raises only the few smallest pivots: the perturbed
    # factors still precondition FGMRES to the target
    rel2 = 1.01 * float(piv.min()) / anorm
    s2 = binding.KKTSolver(pivot_perturb_rel=rel2, **layout)
    s2.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    s2.refactor(dev(vals))
    ora.refactor(vals, perturb_rel=rel2)
    assert_factors_equal(s2.lu()[2], oracle_csr_values(ora))
    b = seq[1][1]
    x = s2.solve(dev(b)).cpu().numpy()
    rep = s2.report()
    print(f"  few perturbed: iters {rep.iters} eta {rep.eta:.3e}", flush=True)
    assert rep.warnings & (1 << binding.WARN_PERTURBED_PIVOT)
    assert eta(pat.scipy(vals), x, b) <= 1e-12


def _tridiag(n, d, o):
    rp = [0]
    ci, v = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
                v.append(d if i == j else o)
        rp.append(len(ci))
    return np.array(rp, np.int64), np.array(ci, np.int32), np.array(v)


def test_reanalysis_restores_a_stable_pivot_order():
    # pivots fixed on a diagonally dominant matrix; the new matrix has a
    # 1e-14 leading entry, so the stored order grows the factors by 1e14 and
    # the direct solve misses the target; re-running the pivoting pass
    # (partial pivoting) swaps the first two rows and the direct solve is exact
    n = 6
    rp, ci, v0 = _tridiag(n, 4.0, 1.0)
    v1 = v0.copy()
    v1[0] = 1e-14
    b = np.random.default_rng(9).standard_normal(n)
    A1 = sp.csr_matrix((v1, ci, rp), shape=(n, n))
    opts = dict(ordering=1, pivot_tau=1.0, fgmres_max_iters=0)
    s = binding.KKTSolver(**opts)
    s.analyze(n, rp, ci, v0)
    s.refactor(dev(v1))
    s.solve(dev(b))
    assert s.report().warnings & (1 << binding.WARN_NOT_CONVERGED)
    s.reanalyze(dev(v1))
    x = s.solve(dev(b)).cpu().numpy()
    assert not s.report().warnings & (1 << binding.WARN_NOT_CONVERGED)
    assert s.last_status == binding.OK and eta(A1, x, b) <= 1e-12
    ora = oracle.OracleLU(n, rp, ci, v1, Q=np.arange(n, dtype=np.int32), tau=1.0)
    assert_factors_equal(s.lu()[2], oracle_csr_values(ora))
    assert not np.array_equal(s.perm()[0], np.arange(n))  # rows were swapped
    # automatic: the solve re-analyses by itself and reports it
    s2 = binding.KKTSolver(auto_reanalyze=1, **opts)
    s2.analyze(n, rp, ci, v0)
    s2.refactor(dev(v1))
    x2 = s2.solve(dev(b)).cpu().numpy()
    assert s2.last_status == binding.OK and eta(A1, x2, b) <= 1e-12
    assert s2.report().warnings & (1 << binding.WARN_REANALYZED)


def test_jacobi_sweeps_truncated_and_exact():
    # approximate triangular solves: k sweeps per triangle.  The GPU's direct
    # solve equals the oracle's truncated sweeps, and as many sweeps as the
    # dependency depth give the exact solve
    pat, seq = kktgen.make_sequence(100, 101, 1)
    vals, b = seq[0]
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, vals, tau=1e-10)

    def sweeps(k):
        return ora.apply_jacobi(b, k)

    A = pat.scipy(vals)
    for k in (3, 12):
        s = binding.KKTSolver(solve_jacobi_sweeps=k, fgmres_max_iters=0)
        s.analyze(pat.n, pat.rowptr, pat.colind, vals)
        s.refactor(dev(vals))
        x = s.solve(dev(b)).cpu().numpy()
        xr = sweeps(k)
        assert np.abs(x - xr).max() <= 1e-9 * np.abs(xr).max(), k
    depth = max(s.info().levels, s.info().levels_u) + 1
    s = binding.KKTSolver(solve_jacobi_sweeps=depth, fgmres_max_iters=0)
    s.analyze(pat.n, pat.rowptr, pat.colind, vals)
    s.refactor(dev(vals))
    x = s.solve(dev(b)).cpu().numpy()
    xo = ora.apply(b)
    assert np.abs(x - xo).max() <= 1e-8 * np.abs(xo).max()
    assert eta(A, x, b) <= 1e-12


def test_jacobi_sweeps_precondition_fgmres():
    # on a well-conditioned matrix a few sweeps are a good enough
    # preconditioner for FGMRES to reach the target
    n = 400
    rp, ci, v = kktgen.random_sparse(n, 0.01, seed=31)
    A = sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()
    A[np.diag_indices(n)] += 4.0 + np.abs(A).sum(1)
    Acsr = sp.csr_matrix(A)
    Acsr.sort_indices()
    b = np.random.default_rng(6).standard_normal(n)
    s = binding.KKTSolver(solve_jacobi_sweeps=4)
    s.analyze(n, Acsr.indptr.astype(np.int64), Acsr.indices.astype(np.int32), Acsr.data)
    s.refactor(dev(Acsr.data))
    x = s.solve(dev(b)).cpu().numpy()
    rep = s.report()
    print(f"  4 sweeps: iters {rep.iters} eta {rep.eta:.3e}", flush=True)
    assert s.last_status == binding.OK and eta(Acsr, x, b) <= 1e-12


def test_gradient_matches_oracle():
    pat, seq = kktgen.make_sequence(100, 101, 1)
    vals, _ = seq[0]
    nrhs = 3
    rng = np.random.default_rng(11)
    Bm = rng.standard_normal((nrhs, pat.n))
    Cm = rng.standard_normal((nrhs, pat.n))
    s = binding.KKTSolver()
    s.analyze(pat.n, pat.rowptr, pat.colind, vals)
    s.refactor(dev(vals))
    x = s.solve(dev(Bm.reshape(-1)))
    lam = s.solve(dev(Cm.reshape(-1)), op="T")
    g = s.grad_values(lam, x).cpu().numpy()
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, vals, tau=1e-10)
    xo, _ = ora.solve(Bm.reshape(-1))
    lo, _ = ora.solve(Cm.reshape(-1), op="T")
    go = ora.grad(lo, xo)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    print(f"  grad rel diff {rel:.3e}", flush=True)
    assert rel <= 1e-6
    # the product itself against the oracle's product of the GPU's solves
    go2 = ora.grad(lam.cpu().numpy(), x.cpu().numpy())
    assert np.allclose(g, go2, rtol=1e-12, atol=1e-14 * np.abs(go2).max())


def test_tiny_pivot_warning_and_report():
    pat, seq = kktgen.make_sequence(100, 101, 1)
    vals, b = seq[0]
    s = binding.KKTSolver(tiny_pivot_rel=1e-6)
    s.analyze(pat.n, pat.rowptr, pat.colind, vals)
    s.refactor(dev(vals))
    rep = s.report()
    assert rep.warnings & (1 << binding.WARN_TINY_PIVOT)
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, vals, tau=1e-10)
    assert ora.refactor(vals, tiny_rel=1e-6) == oracle.WARN_TINY_PIVOT
    A = pat.scipy(vals)
    assert rep.anorm_inf == pytest.approx(abs(A).sum(1).max(), rel=1e-15)
    f = ora.factors()
    d = np.abs(f["Ux"][f["Up"][1:] - 1])
    assert rep.min_pivot == d.min() and rep.max_pivot == d.max()


@pytest.mark.parametrize("B,seed,layout", [(100, 101, dict()), (2000, 104, dict()),
                                           (2000, 104, dict(dense_tail=-1)),
                                           (500, 7, dict(schedule=1))])
def test_growth_matches_oracle(B, seed, layout):
    # growth max|u_ij| / ||A||_inf after each refactorization of a sequence.
    # The numerator is exact on both sides (same factors bit for bit, same
    # maximum); ||A||_inf is a row sum of absolute values whose summation order
    # the definition leaves open (eight lanes per row on the GPU, left to right
    # in the oracle), so the figures agree to a few units in the last place
    pat, seq = kktgen.make_sequence(B, seed, 3)
    s = binding.KKTSolver(**layout)
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, seq[0][0], tau=1e-10)
    for vals, _ in seq[1:]:
        s.refactor(dev(vals))
        rep = s.report()
        ora.refactor(vals)
        rp, ci, lu = s.lu()
        rows = np.repeat(np.arange(pat.n), np.diff(rp))
        umax = np.abs(lu[ci >= rows]).max()
        assert umax == np.abs(ora.factors()["Ux"]).max()
        assert rep.growth == umax / rep.anorm_inf
        print(f"  growth {rep.growth:.6e} (oracle {ora.growth():.6e})", flush=True)
        assert abs(rep.growth - ora.growth()) <= 1e-14 * ora.growth()
    # a non-finite entry: the report (still filled in, growth NaN) comes back
    # with the NONFINITE status
    bad = seq[1][0].copy()
    bad[pat.rowptr[pat.n // 2]] = np.nan
    s.refactor(dev(bad))
    with pytest.raises(binding.KKTError) as err:
        s.report()
    assert err.value.status == binding.ERR_NONFINITE


def test_autograd_backward_refuses_replaced_factors():
    # backward after the solver was refactorized for another system would use
    # the wrong factors: it must raise instead of returning a wrong gradient
    pat, vals = _twin(100, 31)
    s = binding.KKTSolver()
    s.analyze(pat.n, pat.rowptr, pat.colind, vals)
    b = dev(np.random.default_rng(1).standard_normal(pat.n))
    v1 = dev(vals).requires_grad_(True)
    x1 = binding.KKTSolveFn.apply(s, v1, b)
    v2 = dev(vals * 1.5).requires_grad_(True)
    x2 = binding.KKTSolveFn.apply(s, v2, b)
    with pytest.raises(RuntimeError, match="refactorized"):
        x1.sum().backward()
    x2.sum().backward()  # the latest forward still differentiates
    assert torch.isfinite(v2.grad).all()


def test_state_and_argument_errors():
    s = binding.KKTSolver()
    with pytest.raises(binding.KKTError) as ei:
        s.nnz = 4
        s.n = 2
        s.refactor(dev(np.ones(4)))
    assert ei.value.status == binding.ERR_STATE
    pat, seq = kktgen.make_sequence(3, 5, 1)
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    b = dev(seq[0][1])
    with pytest.raises(binding.KKTError) as ei:
        s.solve(b, x=b)
    assert ei.value.status == binding.ERR_INVALID_ARG
    # zero right-hand sides is a no-op
    e = torch.empty(0, dtype=torch.float64, device=DEV)
    s.solve(e)


def test_many_rhs_two_passes():
    pat, seq = kktgen.make_sequence(500, 21, 1)
    vals, _ = seq[0]
    s = binding.KKTSolver()
    s.analyze(pat.n, pat.rowptr, pat.colind, vals)
    s.refactor(dev(vals))
    nr = 33  # crosses the 32-column pass boundary
    Bm = np.random.default_rng(5).standard_normal((nr, pat.n))
    A = pat.scipy(vals)
    for op, M in (("N", A), ("T", A.T.tocsr())):
        X = s.solve(dev(Bm.reshape(-1)), op=op).cpu().numpy().reshape(nr, pat.n)
        etas = [eta(M, X[r], Bm[r]) for r in range(nr)]
        print(f"  {op}: max eta {max(etas):.3e}", flush=True)
        assert max(etas) <= 1e-12


def _twin(B, seed):
    """KKT of the configs' pattern with Sigma clamped to [1e-2, 1e2] and a
    (2,2) block of -1: condition ~1e8, so gradients can be pinned tightly."""
    pat = kktgen.make_kkt(B, seed)
    rng = np.random.default_rng(seed)
    vals = pat.values(np.clip(kktgen.draw_sigma(rng, pat.n_p), 1e-2, 1e2))
    lo = pat.rowptr[pat.n_p]
    vals[lo:] = np.where(pat.colind[lo:] >= pat.n_p, -1.0, vals[lo:])
    return pat, vals


def test_autograd_function_oracle_and_finite_differences():
    pat, vals = _twin(100, 31)
    nrhs = 2
    rng = np.random.default_rng(7)
    Bm = rng.standard_normal((nrhs, pat.n))
    Cm = rng.standard_normal((nrhs, pat.n))
    s = binding.KKTSolver()
    s.analyze(pat.n, pat.rowptr, pat.colind, vals)
    v = dev(vals).requires_grad_(True)
    b = dev(Bm.reshape(-1)).requires_grad_(True)
    x = binding.KKTSolveFn.apply(s, v, b)
    loss = (x * dev(Cm.reshape(-1))).sum()
    loss.backward()
    gv = v.grad.cpu().numpy()
    gb = b.grad.cpu().numpy()
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, vals, tau=1e-10)
    xo, _ = ora.solve(Bm.reshape(-1))
    lo, _ = ora.solve(Cm.reshape(-1), op="T")
    go = ora.grad(lo, xo)
    assert np.linalg.norm(gv - go) / np.linalg.norm(go) <= 1e-9
    assert np.linalg.norm(gb - lo) / np.linalg.norm(lo) <= 1e-9
    # central finite differences of L = sum_r c_r^T A^{-1} b_r (dense, float64)
    A = pat.scipy(vals).toarray()
    rows = np.repeat(np.arange(pat.n), np.diff(pat.rowptr))
    h = 1e-6
    # the difference Lp - Lm cancels all but ~eps |L| / h of the quotient
    # (4e-8 here; the two dense solves' own rounding adds a small factor), so
    # the absolute floor is ten times that
    L0 = np.sum(Cm.T * np.linalg.solve(A, Bm.T))
    floor = 10 * np.finfo(np.float64).eps * abs(L0) / h
    for p in np.random.default_rng(3).choice(pat.nnz, 16, replace=False):
        dA = np.zeros_like(A)
        dA[rows[p], pat.colind[p]] = h
        Lp = np.sum(Cm.T * np.linalg.solve(A + dA, Bm.T))
        Lm = np.sum(Cm.T * np.linalg.solve(A - dA, Bm.T))
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gv[p]) <= 1e-5 * abs(gv[p]) + floor, (p, fd, gv[p], floor)
        # the gradient itself is the oracle's entry by entry
        assert abs(gv[p] - go[p]) <= 1e-9 * np.abs(go).max(), (p, gv[p], go[p])


def _batch_cases():
    """4 instances sharing one B=100 pattern (perturbed W, J and own Sigma)
    plus 3 instances with their own patterns (B = 50, 80, 120)."""
    ga = kktgen.make_batch_group_a(100, 61, 4)
    gb = [(kktgen.make_kkt(B, 6100 + i),) for i, B in enumerate((50, 80, 120))]
    insts = []
    for pat, vals, rhs in ga:
        insts.append((0, pat, vals, rhs))
    patterns = [(ga[0][0].n, ga[0][0].rowptr, ga[0][0].colind, ga[0][1])]
    for i, (pat,) in enumerate(gb):
        rng = np.random.default_rng(i)
        vals = pat.values(kktgen.draw_sigma(rng, pat.n_p))
        patterns.append((pat.n, pat.rowptr, pat.colind, vals))
        insts.append((1 + i, pat, vals, rng.standard_normal(pat.n)))
    return patterns, insts


def _instance_lu(s, t):
    rp, ci, v = s.lu()
    r0, r1 = s.row_offset[t], s.row_offset[t + 1]
    return v[rp[r0]:rp[r1]]


def test_batch_matches_per_instance_oracle():
    patterns, insts = _batch_cases()
    s = binding.KKTSolver()
    s.analyze_batch(patterns, [p for p, *_ in insts])
    vals = np.concatenate([v for _, _, v, _ in insts])
    rhs = np.concatenate([b for *_, b in insts])
    s.refactor(dev(vals))
    x = s.solve(dev(rhs)).cpu().numpy()
    etas = s.batch_eta()
    for t, (p, pat, v, b) in enumerate(insts):
        n0, n1 = s.row_offset[t], s.row_offset[t + 1]
        pn, prp, pci, pv0 = patterns[p]
        ora = oracle.OracleLU(pn, prp, pci, pv0, tau=1e-10)
        ora.refactor(v)
        assert_factors_equal(_instance_lu(s, t), oracle_csr_values(ora))
        e = eta(pat.scipy(v), x[n0:n1], b)
        print(f"  instance {t}: eta {e:.3e} (device {etas[t]:.3e})", flush=True)
        assert e <= 1e-12 and etas[t] <= 1e-12 and abs(etas[t] - e) <= 1e-15


@pytest.mark.parametrize("layout", [dict(), dict(solve_chain=1), dict(solve_chain=-1)],
                         ids=lambda d: "-".join(f"{k}{v}" for k, v in d.items()) or "default")
def test_batch_direct_solve_matches_oracle_apply(layout):
    # no refinement: each instance's block of the batch's direct solve (both
    # operations) against the oracle's direct solve of that instance
    patterns, insts = _batch_cases()
    s = binding.KKTSolver(fgmres_max_iters=0, **layout)
    s.analyze_batch(patterns, [p for p, *_ in insts])
    vals = np.concatenate([v for _, _, v, _ in insts])
    rhs = np.concatenate([b for *_, b in insts])
    s.refactor(dev(vals))
    for op in ("N", "T"):
        x = s.solve(dev(rhs), op=op).cpu().numpy()
        for t, (p, pat, v, b) in enumerate(insts):
            n0, n1 = s.row_offset[t], s.row_offset[t + 1]
            pn, prp, pci, pv0 = patterns[p]
            ora = oracle.OracleLU(pn, prp, pci, pv0, tau=1e-10)
            ora.refactor(v)
            xo = ora.apply(b, op)
            err = np.abs(x[n0:n1] - xo).max() / np.abs(xo).max()
            assert err <= 1e-8, (layout, op, t, err)


def test_graph_replay_matches_eager():
    patterns, insts = _batch_cases()
    s = binding.KKTSolver()
    s.analyze_batch(patterns, [p for p, *_ in insts])
    rng = np.random.default_rng(17)
    stream = torch.cuda.Stream()
    base_v = np.concatenate([v for _, _, v, _ in insts])
    vbuf = dev(base_v)
    bbuf = dev(np.concatenate([b for *_, b in insts]))
    xbuf = torch.empty_like(bbuf)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        s.graph_capture(vbuf, bbuf, xbuf, stream)
    stream.synchronize()
    ref = binding.KKTSolver()
    ref.analyze_batch(patterns, [p for p, *_ in insts])
    for rep in range(4):
        # new Sigma-like diagonal scaling per replay, written into the captured buffers
        v_new = base_v * (1.0 + 0.01 * rng.standard_normal(base_v.size))
        b_new = rng.standard_normal(bbuf.numel())
        vbuf.copy_(dev(v_new))
        bbuf.copy_(dev(b_new))
        torch.cuda.synchronize()
        s.graph_launch(stream)
        stream.synchronize()
        # eager reference on another handle, with a host synchronisation between replays
        ref.refactor(dev(v_new))
        x_ref = ref.solve(dev(b_new)).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(s.lu()[2].view(np.int64), ref.lu()[2].view(np.int64))
        xg = xbuf.cpu().numpy()
        etas = s.batch_eta()
        print(f"  replay {rep}: max eta {etas.max():.3e}", flush=True)
        assert etas.max() <= 1e-12
        assert np.allclose(xg, x_ref, rtol=1e-9, atol=1e-12 * np.abs(x_ref).max())


def test_graph_replays_refine_on_the_device():
    # static pivoting raises the pivots below 1e-11 ||A||: the captured
    # refactorization's factors are those of a nearby matrix and every replay
    # needs several FGMRES iterations, all inside the graph (no host step)
    pat, seq = kktgen.make_sequence(500, 7, 4)
    s = binding.KKTSolver(pivot_perturb_rel=1e-11, fgmres_max_iters=40)
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    stream = torch.cuda.Stream()
    vbuf = dev(seq[1][0])
    bbuf = dev(seq[1][1])
    xbuf = torch.empty_like(bbuf)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        s.graph_capture(vbuf, bbuf, xbuf, stream)
    stream.synchronize()
    for k in (1, 2, 3, 1):
        vals, b = seq[k]
        vbuf.copy_(dev(vals))
        bbuf.copy_(dev(b))
        torch.cuda.synchronize()
        s.graph_launch(stream)
        stream.synchronize()
        rep = s.report()
        x = xbuf.cpu().numpy()
        e = eta(pat.scipy(vals), x, b)
        print(f"  replay of step {k}: iters {rep.iters} eta0 {rep.eta0:.3e} eta {e:.3e}", flush=True)
        assert rep.iters >= 1 and rep.eta0 > 1e-12
        assert e <= 1e-12 and rep.eta <= 1e-12
        assert not rep.warnings & (1 << binding.WARN_NOT_CONVERGED)


def test_batch_graph_forced_iterations():
    # two forced FGMRES iterations on the block-diagonal batch, captured
    patterns, insts = _batch_cases()
    s = binding.KKTSolver(min_iters=2)
    s.analyze_batch(patterns, [p for p, *_ in insts])
    stream = torch.cuda.Stream()
    vbuf = dev(np.concatenate([v for _, _, v, _ in insts]))
    bbuf = dev(np.concatenate([b for *_, b in insts]))
    xbuf = torch.empty_like(bbuf)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        s.graph_capture(vbuf, bbuf, xbuf, stream)
    for _ in range(3):
        s.graph_launch(stream)
    stream.synchronize()
    rep = s.report()
    etas = s.batch_eta()
    x = xbuf.cpu().numpy()
    assert rep.iters == 2 and etas.max() <= 1e-12
    for t, (p, pat, v, b) in enumerate(insts):
        n0, n1 = s.row_offset[t], s.row_offset[t + 1]
        assert eta(pat.scipy(v), x[n0:n1], b) <= 1e-12, t


@pytest.mark.parametrize("op", ["N", "T"])
def test_multi_rhs_device_refinement_stale(op):
    # eleven right-hand sides (a group of eight and a group of three refined
    # in lockstep) against factors of a 5 %-perturbed matrix
    pat = kktgen.make_kkt(500, 77)
    rng = np.random.default_rng(3)
    sigma = np.clip(kktgen.draw_sigma(rng, pat.n_p), 1e-2, 1e2)
    v_old = pat.values(sigma)
    sym = pat.scipy(v_old * (1.0 + 0.05 * rng.standard_normal(v_old.size)))
    sym = (sym + sym.T) * 0.5
    sym.sort_indices()
    v_new = sym.data
    nrhs = 11
    B = rng.standard_normal((nrhs, pat.n))
    s = binding.KKTSolver()
    s.analyze(pat.n, pat.rowptr, pat.colind, v_old)
    s.refactor(dev(v_old))
    s.update_matrix(dev(v_new))
    X = s.solve(dev(B.reshape(-1)), op=op).cpu().numpy().reshape(nrhs, pat.n)
    rep = s.report()
    M = pat.scipy(v_new) if op == "N" else pat.scipy(v_new).T.tocsr()
    etas = [eta(M, X[r], B[r]) for r in range(nrhs)]
    print(f"  op {op}: iters {rep.iters} max eta {max(etas):.3e}", flush=True)
    assert rep.iters > 1 and max(etas) <= 1e-12 and rep.eta <= 1e-12


def test_multi_rhs_forced_iterations_wide_grid():
    # eight right-hand sides refined in lockstep on a system of about 70k
    # rows with two forced iterations: the Arnoldi pass then runs on its
    # widest grid, whose per-workgroup partial sums for eight columns must
    # stay inside their buffer (the residual pass may use a wider grid)
    pat, seq = kktgen.make_sequence(7000, 107, 1)
    vals, _ = seq[0]
    nrhs = 8
    B = np.random.default_rng(5).standard_normal((nrhs, pat.n))
    s = binding.KKTSolver(min_iters=2)
    s.analyze(pat.n, pat.rowptr, pat.colind, vals)
    s.refactor(dev(vals))
    X = s.solve(dev(B.reshape(-1))).cpu().numpy().reshape(nrhs, pat.n)
    rep = s.report()
    A = pat.scipy(vals)
    etas = [eta(A, X[r], B[r]) for r in range(nrhs)]
    print(f"  n {pat.n}: iters {rep.iters} max eta {max(etas):.3e}", flush=True)
    assert pat.n > 512 * 128 and rep.iters == 2 and max(etas) <= 1e-12


def test_adaptive_refinement_budget():
    # refine_budget = -1: exact factors need no iteration, so later solves
    # launch two; kkt_update_matrix (stale factors) brings the full budget
    # back, and a later solve on the same stale factors launches enough for
    # the iterations its predecessor needed
    pat = kktgen.make_kkt(500, 77)
    rng = np.random.default_rng(3)
    sigma = np.clip(kktgen.draw_sigma(rng, pat.n_p), 1e-2, 1e2)
    v_old = pat.values(sigma)
    sym = pat.scipy(v_old * (1.0 + 0.05 * rng.standard_normal(v_old.size)))
    sym = (sym + sym.T) * 0.5
    sym.sort_indices()
    v_new = sym.data
    b = rng.standard_normal(pat.n)
    s = binding.KKTSolver(refine_budget=-1)
    s.analyze(pat.n, pat.rowptr, pat.colind, v_old)
    for _ in range(3):
        s.refactor(dev(v_old))
        x = s.solve(dev(b)).cpu().numpy()
        rep = s.report()
        assert rep.iters == 0 and eta(pat.scipy(v_old), x, b) <= 1e-12
    s.update_matrix(dev(v_new))
    its = []
    for _ in range(2):
        x = s.solve(dev(b)).cpu().numpy()
        torch.cuda.synchronize()
        rep = s.report()
        its.append(rep.iters)
        assert not rep.warnings & (1 << binding.WARN_NOT_CONVERGED)
        assert eta(pat.scipy(v_new), x, b) <= 1e-12
    print(f"  stale solves: iters {its}", flush=True)
    assert its[0] > 2 and its[1] == its[0]


def test_solve_does_not_wait_for_the_device():
    # a long spin kernel ahead on the stream: refactor and solve return while
    # it still runs (no host synchronisation), and the result is right after
    if not hasattr(torch.cuda, "_sleep"):
        pytest.skip("torch.cuda._sleep unavailable")
    pat, seq = kktgen.make_sequence(100, 101, 2)
    vals, b = seq[1]
    s = binding.KKTSolver()
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    vd, bd = dev(vals), dev(b)
    x = torch.empty_like(bd)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    torch.cuda._sleep(200_000_000)
    s.refactor(vd)
    s.solve(bd, x)
    busy = not stream.query()
    torch.cuda.synchronize()
    assert busy, "kkt_solve waited for the device"
    assert eta(pat.scipy(vals), x.cpu().numpy(), b) <= 1e-12


@pytest.mark.parametrize("B,seed", [(500, 7), (2000, 104)])
def test_adversarial_schedule_bitwise(B, seed):
    # another workgroup (and XCD) for every chunk of the persistent kernels
    # and pseudo-random pauses after each fetch: the factors are still the
    # oracle's bit for bit and the solve meets the target
    pat, seq = kktgen.make_sequence(B, seed, 2)
    vals, b = seq[1]
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, seq[0][0], tau=1e-10)
    ora.refactor(vals)
    s = binding.KKTSolver(debug_schedule=1)
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    for _ in range(2):
        s.refactor(dev(vals))
        x = s.solve(dev(b)).cpu().numpy()
        assert_factors_equal(s.lu()[2], oracle_csr_values(ora))
        assert eta(pat.scipy(vals), x, b) <= 1e-12
    s.close()
    # the flag is process-wide: the next analysis restores the plain schedule
    r = binding.KKTSolver()
    r.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    r.close()


def test_tiny_spin_limit_drains_and_reports():
    # every dependency wait gives up on its second poll: the kernels run to
    # their end (no hang), the stall flag is raised and the report says so
    pat, seq = kktgen.make_sequence(2000, 104, 2)
    vals, b = seq[1]
    s = binding.KKTSolver(debug_spin_limit=1)
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    s.refactor(dev(vals))
    s.solve(dev(b))
    torch.cuda.synchronize()
    with pytest.raises(binding.KKTError) as err:
        s.report()
    assert err.value.status == binding.ERR_DEVICE
    s.close()


@pytest.mark.parametrize("layout", [dict(), dict(schedule=1), dict(schedule=2, sync_mode=1),
                                    dict(solve_chain=-1), dict(dense_tail=300)],
                         ids=["default", "levels", "fences", "level-chunks", "dense-block"])
def test_matching_and_scaling_bitwise(layout):
    # matched and scaled analysis (Section 5.2.1): the product's matching and
    # power-of-two scaling equal the oracle's, every refactorization of the
    # sequence gives the oracle's factors of Ahat = Pm Dr A Dc bit for bit,
    # and the solves of A (both ops, several right-hand sides) meet the target
    pat, seq = kktgen.make_sequence(100, 101, 3)
    s = binding.KKTSolver(matching=1, **layout)
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    m, dr, dc = s.scaling()
    m0, dr0, dc0 = oracle.match_scale(pat.n, pat.rowptr, pat.colind, seq[0][0])
    assert np.array_equal(m, m0) and np.array_equal(dr, dr0) and np.array_equal(dc, dc0)
    hrp, hci, hv, src = oracle.matched_scaled(pat.n, pat.rowptr, pat.colind, seq[0][0], m, dr, dc)
    ora = oracle.OracleLU(pat.n, hrp, hci, hv, tau=1e-10)
    assert not np.array_equal(m, np.arange(pat.n)), "the matching should permute rows here"
    for vals, b in seq[1:]:
        s.refactor(dev(vals))
        ora.refactor(dr[m][np.repeat(np.arange(pat.n), np.diff(hrp))] * vals[src] * dc[hci])
        assert_factors_equal(s.lu()[2], oracle_csr_values(ora))
        A = pat.scipy(vals)
        x = s.solve(dev(b)).cpu().numpy()
        assert eta(A, x, b) <= 1e-12
        lam = s.solve(dev(b), op="T").cpu().numpy()
        assert eta(A.T.tocsr(), lam, b) <= 1e-12
    B3 = np.random.default_rng(5).standard_normal((3, pat.n))
    X = s.solve(dev(B3.reshape(-1))).cpu().numpy().reshape(3, pat.n)
    for r in range(3):
        assert eta(A, X[r], B3[r]) <= 1e-12
    # a re-analysis keeps the matching and scaling
    s.reanalyze(dev(seq[2][0]))
    m2, dr2, dc2 = s.scaling()
    assert np.array_equal(m2, m) and np.array_equal(dr2, dr)
    x = s.solve(dev(seq[2][1])).cpu().numpy()
    assert eta(pat.scipy(seq[2][0]), x, seq[2][1]) <= 1e-12


def test_autotuner_picks_a_working_schedule(tmp_path):
    from paper_2306_14337_amd import autotune

    pat, seq = kktgen.make_sequence(500, 12, 1)
    vals, b = seq[0]
    cache = str(tmp_path / "tune.json")
    best, times = autotune.autotune(pat.n, pat.rowptr, pat.colind, vals, dev(vals), dev(b),
                                    repeats=1, cache_path=cache)
    print(f"  best {best}, {len(times)} candidates timed", flush=True)
    assert len(times) >= 2
    s = binding.KKTSolver(**best)
    s.analyze(pat.n, pat.rowptr, pat.colind, vals)
    s.refactor(dev(vals))
    x = s.solve(dev(b)).cpu().numpy()
    assert eta(pat.scipy(vals), x, b) <= 1e-12
    again, t2 = autotune.autotune(pat.n, pat.rowptr, pat.colind, vals, dev(vals), dev(b),
                                  cache_path=cache)
    assert again == best and t2 == {}


def test_batch_autotuner_picks_working_knobs(tmp_path):
    from paper_2306_14337_amd import autotune

    patterns, insts = _batch_cases()
    inst_pattern = [p for p, *_ in insts]
    vals = dev(np.concatenate([v for _, _, v, _ in insts]))
    rhs = np.concatenate([b for *_, b in insts])
    cache = str(tmp_path / "tune.json")
    best, times = autotune.autotune_batch(patterns, inst_pattern, vals, dev(rhs), repeats=1,
                                          cache_path=cache)
    print(f"  best {best}, times {times}", flush=True)
    assert len(times) >= 2 and "{}" in times
    # the winner runs the batch to the target, factors bitwise as the defaults
    s = binding.KKTSolver(**best)
    s.analyze_batch(patterns, inst_pattern)
    s.refactor(vals)
    x = s.solve(dev(rhs)).cpu().numpy()
    ref = binding.KKTSolver()
    ref.analyze_batch(patterns, inst_pattern)
    ref.refactor(vals)
    assert np.array_equal(s.lu()[2].view(np.int64), ref.lu()[2].view(np.int64))
    for t, (p, pat, v, b) in enumerate(insts):
        n0, n1 = s.row_offset[t], s.row_offset[t + 1]
        assert eta(pat.scipy(v), x[n0:n1], b) <= 1e-12, t
    again, t2 = autotune.autotune_batch(patterns, inst_pattern, vals, dev(rhs), cache_path=cache)
    assert again == best and t2 == {}


def test_row_timeline_records_every_band_row():
    # debug_timeline: every row the two band kernels take is stamped, its
    # start precedes its end, no row ends before an input it read, and the
    # factors are the oracle's as without the recording
    from paper_2306_14337_amd import timeline

    pat, seq = kktgen.make_sequence(2000, 104, 2)
    s = binding.KKTSolver(debug_timeline=1)
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    vals, _ = seq[1]
    s.refactor(dev(vals))
    tl = s.debug_timeline()
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, seq[0][0], tau=1e-10)
    ora.refactor(vals)
    assert_factors_equal(s.lu()[2], oracle_csr_values(ora))
    rp, ci, _ = s.lu(values=False)
    c0 = pat.n - int(s.info().dense_tail)
    rec = tl[:, 3] > 0
    rows = np.repeat(np.arange(pat.n), np.diff(rp))
    # rows with a pivot before the dense block go through a band kernel
    has_piv = np.zeros(pat.n, bool)
    has_piv[rows[(ci < rows) & (ci < c0)]] = True
    print(f"  recorded {rec.sum()} rows, kinds {np.bincount(tl[:, 3], minlength=4)}", flush=True)
    assert np.array_equal(rec, has_piv)
    assert set(np.unique(tl[rec, 3])) <= {1, 2, 3}
    assert (tl[rec, 0] <= tl[rec, 1]).all() and (tl[rec, 1] <= tl[rec, 2]).all()
    # causality: a recorded input made its values after its last poll that
    # still found one of its own inputs missing, and the row needed those
    # values, so the row ended after that poll (2 us of clock slack).  The
    # input's own end stamp follows its wait for the store acknowledgements
    # and may come later than a reader's end.
    dep = (ci < rows) & rec[rows] & rec[np.minimum(ci, pat.n - 1)] & (ci < c0)
    assert (tl[rows[dep], 2] >= tl[ci[dep], 1] - 2000).all()
    chain = timeline.critical_chain(tl, rp, ci)
    assert len(chain) >= 2 and tl[chain[-1], 2] == tl[rec, 2].max()
    print(timeline.summary(tl, rp, ci, c0), flush=True)
    s.close()
    with pytest.raises(binding.KKTError):
        plain = binding.KKTSolver()
        plain.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
        plain.debug_timeline()


def test_nonfinite_values_are_reported_not_waited_on():
    # a refactorization whose values hold a NaN -- including one with the bit
    # pattern the kernels use for "not yet computed" -- finishes and reports
    # NONFINITE; a right-hand side with that pattern is solved (to NaNs) too
    pat, seq = kktgen.make_sequence(100, 101, 2)
    vals, b = seq[1]
    s = binding.KKTSolver()
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    sentinel = np.array([0x7FF0DEAD5EED0001], dtype=np.uint64).view(np.float64)[0]
    for bad in (sentinel, np.nan, np.inf):
        v = vals.copy()
        v[len(v) // 2] = bad
        s.refactor(dev(v))
        torch.cuda.synchronize()
        with pytest.raises(binding.KKTError) as err:
            s.report()
        assert err.value.status == binding.ERR_NONFINITE, bad
    s.refactor(dev(vals))
    x = s.solve(dev(b)).cpu().numpy()
    assert s.report().eta <= 1e-12 and eta(pat.scipy(vals), x, b) <= 1e-12
    bb = b.copy()
    bb[3] = sentinel
    x = s.solve(dev(bb)).cpu().numpy()
    rep = s.report()
    assert rep.warnings & (1 << binding.WARN_NOT_CONVERGED) and np.isnan(x).any()
