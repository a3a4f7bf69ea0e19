"""kkt_solve_noalloc (scratch in the library's static device array) against
kkt_solve (scratch in the handle's workspace), through the C ABI.

Two calls in a row on one GPU, the second with a smaller input: eleven
right-hand sides of a 500-bus system whose factors are stale (so the
refinement state in the scratch array is exercised over several
iterations), then two right-hand sides of a 100-bus system.  Both entry
points run the same kernels on the same inputs, so the solutions must agree
to the solve's accuracy bar (and in practice bit for bit).
"""
import numpy as np
import pytest

from paper_2306_14337_amd import binding, kktgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def eta(A, x, b):
    return np.abs(b - A @ x).max() / (abs(A).sum(1).max() * np.abs(x).max())


def _stale_case(B, seed, nrhs):
    pat = kktgen.make_kkt(B, seed)
    rng = np.random.default_rng(seed)
    sigma = np.clip(kktgen.draw_sigma(rng, pat.n_p), 1e-2, 1e2)
    v_old = pat.values(sigma)
    sym = pat.scipy(v_old * (1.0 + 0.05 * rng.standard_normal(v_old.size)))
    sym = (sym + sym.T) * 0.5
    sym.sort_indices()
    return pat, v_old, sym.data, rng.standard_normal(nrhs * pat.n)


def test_noalloc_solve_matches_solve_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for B, seed, nrhs, op in ((500, 81, 11, "N"), (100, 82, 2, "T")):
        pat, v_old, v_new, b = _stale_case(B, seed, nrhs)
        s = binding.KKTSolver()
        s.analyze(pat.n, pat.rowptr, pat.colind, v_old)
        s.refactor(dev(v_old))
        s.update_matrix(dev(v_new))
        bd = dev(b)
        x_ref = s.solve(bd, op=op).cpu().numpy()
        rep_ref = s.report()
        x_na = torch.empty_like(bd)
        s.solve_noalloc(bd, x_na, op=op)
        rep_na = s.report()
        x_na = x_na.cpu().numpy()
        M = pat.scipy(v_new) if op == "N" else pat.scipy(v_new).T.tocsr()
        X = x_na.reshape(nrhs, pat.n)
        Bm = b.reshape(nrhs, pat.n)
        e = max(eta(M, X[r], Bm[r]) for r in range(nrhs))
        same = np.array_equal(x_na.view(np.int64), x_ref.view(np.int64))
        print(f"\n  B={B} nrhs={nrhs} op={op}: iters {rep_na.iters} (kkt_solve {rep_ref.iters}) "
              f"eta {e:.3e} bitwise {same}", flush=True)
        assert rep_na.iters == rep_ref.iters and rep_na.iters > 1
        assert rep_na.eta <= 1e-12 and e <= 1e-12
        assert np.abs(x_na - x_ref).max() <= 1e-12 * np.abs(x_ref).max()
        s.close()
