"""GPU path vs the CPU oracle at the sizes of the adjoint and batched workloads.

* Adjoint: B = 10,000 buses (n = 99,996), 32 right-hand sides, loss
  L = sum_r c_r . x_r.  Backward errors of every x_r and lambda_r, the GPU
  gradient on the pattern against the oracle's, and a central difference
  with h = 1e-6 on 64 seeded stored entries, on the generator's matrix and on
  a well-conditioned twin (Sigma clamped to [1e-2, 1e2]).
* Batched: instances of a shared B = 2,000 pattern and an instance with its
  own B = 5,000 pattern in one block-diagonal batch; every instance's factors
  bit for bit against the oracle, and per-instance eta.

Central difference.  For a stored entry p = (i, j) and E = e_i e_j^T, the
quotient is q = sum_r c_r . (x_r(+h) - x_r(-h)) / (2h) with (A +- hE) x(+-h) =
b.  The two solutions agree to ~h |x| while each carries rounding of order
kappa u |x| (kappa ~ 1e16 here), so their difference is formed by one more
solve instead of a subtraction: (A + hE)(x(+h) - x(-h)) = -2h E x(-h) exactly,
hence x(+h) - x(-h) = -2h x(-h)_j (A + hE)^{-1} e_i.  Both matrices are
refactorized by the oracle; nothing is linearized.  Since E has rank one,
q = g / (1 - h^2 a^2) with a = (A^{-1})_ji, so an entry with h |a| > 1e-2 is
reported as FD-invalid (its quotient is not within 1e-4 of the derivative)
and left out; the count is printed.
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


@pytest.mark.parametrize("twin", [False, True], ids=["kappa~1e16", "clamped-sigma"])
def test_adjoint_at_10k_buses_32_rhs(twin):
    B, seed, nrhs = 10000, 105, 32
    pat = kktgen.make_kkt(B, seed)
    sigma = kktgen.draw_sigma(np.random.default_rng(seed * 10), pat.n_p)
    if twin:
        sigma = np.clip(sigma, 1e-2, 1e2)
    vals = pat.values(sigma)
    Bm = np.random.default_rng(seed * 10 + 2).standard_normal(nrhs * pat.n)
    Cm = np.random.default_rng(seed * 10 + 1).standard_normal(nrhs * pat.n)
    n = pat.n
    print(f"\n  n={n} nnz={pat.nnz} nrhs={nrhs} twin={twin}", flush=True)
    # GPU: forward, transposed solve with the same factors, gradient
    s = binding.KKTSolver()
    s.analyze(n, pat.rowptr, pat.colind, vals)
    s.refactor(dev(vals))
    x = s.solve(dev(Bm))
    lam = s.solve(dev(Cm), op="T")
    g = s.grad_values(lam, x).cpu().numpy()
    X = x.cpu().numpy().reshape(nrhs, n)
    Lm = lam.cpu().numpy().reshape(nrhs, n)
    A = pat.scipy(vals)
    At = A.T.tocsr()
    ex = max(eta(A, X[r], Bm[r * n:(r + 1) * n]) for r in range(nrhs))
    el = max(eta(At, Lm[r], Cm[r * n:(r + 1) * n]) for r in range(nrhs))
    print(f"  eta max: x {ex:.3e}, lambda {el:.3e}", flush=True)
    assert ex <= 1e-12 and el <= 1e-12
    # the oracle's gradient from its own solves
    ora = oracle.OracleLU(n, pat.rowptr, pat.colind, vals, tau=1e-10)
    xo, _ = ora.solve(Bm)
    lo, _ = ora.solve(Cm, op="T")
    go = ora.grad(lo, xo)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    print(f"  gradient vs oracle: rel {rel:.3e} (growth {ora.growth():.3e})", flush=True)
    assert rel <= (1e-9 if twin else 1e-6)
    # central differences on 64 seeded stored entries (oracle evaluations)
    rows = np.repeat(np.arange(n), np.diff(pat.rowptr))
    C2 = Cm.reshape(nrhs, n)
    h = 1e-6
    rtol = 1e-5 if twin else 1e-4
    floor = 1e-12 * np.abs(g).max()
    invalid, worst = 0, 0.0
    for p in np.random.default_rng(seed * 10 + 3).choice(pat.nnz, 64, replace=False):
        i, j = int(rows[p]), int(pat.colind[p])
        e = np.zeros(n)
        e[i] = 1.0
        ora.refactor(vals)
        a = ora.apply(e)[j]
        if h * abs(a) > 1e-2:
            invalid += 1
            continue
        vm = vals.copy()
        vm[p] -= h
        ora.refactor(vm)
        xm, _ = ora.solve(Bm)
        vp = vals.copy()
        vp[p] += h
        ora.refactor(vp)
        w, _ = ora.solve(e)
        q = -float((C2 @ w) @ xm.reshape(nrhs, n)[:, j])
        err = abs(q - g[p])
        worst = max(worst, err / (abs(g[p]) + floor))
        assert err <= rtol * abs(g[p]) + floor, (int(p), q, g[p])
    print(f"  central differences: {64 - invalid} checked, {invalid} FD-invalid, "
          f"worst rel {worst:.3e}", flush=True)
    assert invalid <= 16


def test_batch_with_2000_and_5000_bus_instances():
    # two instances of a shared B = 2,000 pattern (perturbed W, J, own Sigma)
    # and one B = 5,000 instance with its own pattern: rows long enough for
    # the long-row refactorization band in batch mode
    ga = kktgen.make_batch_group_a(2000, 104, 2)
    pb = kktgen.make_kkt(5000, 104 * 1000)
    rng = np.random.default_rng(104 * 100000)
    vb = pb.values(kktgen.draw_sigma(rng, pb.n_p))
    bb = rng.standard_normal(pb.n)
    insts = [(0, p, v, r) for p, v, r in ga] + [(1, pb, vb, bb)]
    patterns = [(ga[0][0].n, ga[0][0].rowptr, ga[0][0].colind, ga[0][1]),
                (pb.n, pb.rowptr, pb.colind, vb)]
    s = binding.KKTSolver()
    s.analyze_batch(patterns, [p for p, *_ in insts])
    vals = np.concatenate([v for _, _, v, _ in insts])
    rhs = np.concatenate([r for *_, r in insts])
    s.refactor(dev(vals))
    x = s.solve(dev(rhs)).cpu().numpy()
    etas = s.batch_eta()
    rp, _, lu = s.lu()
    for t, (p, pat, v, b) in enumerate(insts):
        r0, r1 = s.row_offset[t], s.row_offset[t + 1]
        pn, prp, pci, pv0 = patterns[p]
        ora = oracle.OracleLU(pn, prp, pci, pv0, tau=1e-10)
        ora.refactor(v)
        ov = oracle_csr_values(ora)
        gv = lu[rp[r0]:rp[r1]]
        longest = int(np.diff(rp[r0:r1 + 1]).max())
        print(f"  instance {t}: n={pn} factor entries {len(ov)} longest row {longest}", flush=True)
        assert np.array_equal(gv.view(np.int64), ov.view(np.int64)), (
            f"instance {t}: {np.sum(gv != ov)} factor entries differ")
        e = eta(pat.scipy(v), x[r0:r1], b)
        print(f"  instance {t}: eta {e:.3e} (device {etas[t]:.3e})", flush=True)
        assert e <= 1e-12 and etas[t] <= 1e-12
    assert int(np.diff(rp).max()) > 128, "no row reached the long-row band"
