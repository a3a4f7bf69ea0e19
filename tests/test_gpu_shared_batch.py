"""Shared-pattern batches (kkt_analyze_shared) on the GPU, through the C ABI.

count instances of one pattern share one analysis and one copy of every index
structure; each instance has its own values and vectors.  Checks:
* factors of every instance equal the oracle's refactorization of that
  instance bit for bit, and equal the block-diagonal batch of the same
  instances (kkt_analyze_batch), whose kernels take every instance's rows as
  rows of one merged system;
* direct solves (no refinement) match the oracle's per instance, both
  operations; refined solves and graph replays with forced iterations meet
  eta <= 1e-12 per instance;
* the calls a shared batch does not support fail with their documented status.
"""
import numpy as np
import pytest

import oracle
from paper_2306_14337_amd import binding, kktgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def eta(A, x, b):
    return np.abs(b - A @ x).max() / (abs(A).sum(1).max() * np.abs(x).max())


def oracle_csr_values(lu):
    f = lu.factors()
    n = lu.n
    rows = np.concatenate([f["Li"], f["Ui"]])
    cols = np.concatenate([np.repeat(np.arange(n), np.diff(f["Lp"])),
                           np.repeat(np.arange(n), np.diff(f["Up"]))])
    vals = np.concatenate([f["Lx"], f["Ux"]])
    return vals[np.lexsort((cols, rows))]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()
    yield


def _instances(B, seed, count):
    """count instances of one pattern (own W, J perturbation and Sigma each)."""
    ga = kktgen.make_batch_group_a(B, seed, count)
    pat = ga[0][0]
    return pat, [v for _, v, _ in ga], [r for _, _, r in ga]


@pytest.mark.parametrize("B,seed,count", [(3, 5, 3), (100, 61, 5), (2000, 104, 6)])
def test_shared_factors_bitwise(B, seed, count):
    print(f"case B={B} seed={seed} count={count}", flush=True)
    pat, vals, _ = _instances(B, seed, count)
    s = binding.KKTSolver()
    s.analyze_shared(pat.n, pat.rowptr, pat.colind, vals[0], count)
    assert s.n == pat.n * count and s.count == count
    allv = np.concatenate(vals)
    s.refactor(dev(allv))
    rp, ci, lv = s.lu()
    f = len(lv) // count
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, vals[0], tau=1e-10)
    for t in range(count):
        ora.refactor(vals[t])
        got = lv[t * f:(t + 1) * f]
        want = oracle_csr_values(ora)
        assert np.array_equal(got.view(np.int64), want.view(np.int64)), (
            t, int(np.sum(got != want)))
    # the block-diagonal batch of the same instances: the same factors and
    # the same block-diagonal pattern
    bd = binding.KKTSolver()
    bd.analyze_batch([(pat.n, pat.rowptr, pat.colind, vals[0])], [0] * count)
    bd.refactor(dev(allv))
    rp2, ci2, lv2 = bd.lu()
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2)
    assert np.array_equal(lv.view(np.int64), lv2.view(np.int64))
    assert s.info().nnz == pat.nnz * count


@pytest.mark.parametrize("op", ["N", "T"])
def test_shared_direct_solve_matches_oracle(op):
    pat, vals, rhs = _instances(100, 61, 5)
    count = len(vals)
    s = binding.KKTSolver(fgmres_max_iters=0)
    s.analyze_shared(pat.n, pat.rowptr, pat.colind, vals[0], count)
    s.refactor(dev(np.concatenate(vals)))
    x = s.solve(dev(np.concatenate(rhs)), op=op).cpu().numpy()
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, vals[0], tau=1e-10)
    for t in range(count):
        ora.refactor(vals[t])
        xo = ora.apply(rhs[t], op)
        xt = x[t * pat.n:(t + 1) * pat.n]
        err = np.abs(xt - xo).max() / np.abs(xo).max()
        assert err <= 1e-8, (op, t, err)


@pytest.mark.parametrize("op", ["N", "T"])
def test_shared_refined_solve_per_instance(op):
    pat, vals, rhs = _instances(2000, 104, 6)
    count = len(vals)
    s = binding.KKTSolver(min_iters=2)
    s.analyze_shared(pat.n, pat.rowptr, pat.colind, vals[0], count)
    s.refactor(dev(np.concatenate(vals)))
    x = s.solve(dev(np.concatenate(rhs)), op=op).cpu().numpy()
    rep = s.report()
    etas = s.batch_eta()
    print(f"  op {op}: iters {rep.iters} max eta {etas.max():.3e}", flush=True)
    assert rep.iters == 2 and etas.max() <= 1e-12
    for t in range(count):
        A = pat.scipy(vals[t])
        M = A if op == "N" else A.T.tocsr()
        e = eta(M, x[t * pat.n:(t + 1) * pat.n], rhs[t])
        assert e <= 1e-12 and abs(e - etas[t]) <= 1e-15, (t, e, etas[t])


def test_shared_graph_replays():
    # refactorization, solve and device-checked refinement (two forced
    # iterations) captured once and replayed with new values each time
    pat, vals, rhs = _instances(500, 7, 4)
    count = len(vals)
    rng = np.random.default_rng(9)
    s = binding.KKTSolver(min_iters=2)
    s.analyze_shared(pat.n, pat.rowptr, pat.colind, vals[0], count)
    base = np.concatenate(vals)
    vbuf = dev(base)
    bbuf = dev(np.concatenate(rhs))
    xbuf = torch.empty_like(bbuf)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    s.graph_capture(vbuf, bbuf, xbuf, stream)
    stream.synchronize()
    for rep_i in range(3):
        v_new = base * (1.0 + 0.01 * rng.standard_normal(base.size))
        vbuf.copy_(dev(v_new))
        torch.cuda.synchronize()
        s.graph_launch(stream)
        stream.synchronize()
        x = xbuf.cpu().numpy()
        etas = s.batch_eta()
        print(f"  replay {rep_i}: max eta {etas.max():.3e}", flush=True)
        assert etas.max() <= 1e-12
        for t in range(count):
            A = pat.scipy(v_new[t * pat.nnz:(t + 1) * pat.nnz])
            assert eta(A, x[t * pat.n:(t + 1) * pat.n], rhs[t]) <= 1e-12, (rep_i, t)


def test_shared_unsupported_calls():
    pat, vals, rhs = _instances(100, 61, 3)
    count = len(vals)
    with pytest.raises(binding.KKTError) as err:
        binding.KKTSolver(matching=1).analyze_shared(pat.n, pat.rowptr, pat.colind, vals[0], count)
    assert err.value.status == binding.ERR_INVALID_ARG
    s = binding.KKTSolver()
    s.analyze_shared(pat.n, pat.rowptr, pat.colind, vals[0], count)
    s.refactor(dev(np.concatenate(vals)))
    b = dev(np.concatenate(rhs))
    with pytest.raises(binding.KKTError) as err:
        s.solve(torch.cat([b, b]))  # two right-hand sides per instance
    assert err.value.status == binding.ERR_INVALID_ARG
    x = s.solve(b)
    lam = s.solve(b, op="T")
    g = torch.empty(pat.nnz * count, dtype=torch.float64, device=DEV)
    with pytest.raises(binding.KKTError) as err:
        s.grad_values(lam, x, g)
    assert err.value.status == binding.ERR_STATE
