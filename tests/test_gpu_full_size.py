"""The 70k-bus workload at full size, in the launch configuration the benchmark
times (library defaults), vs the CPU oracle (needs an MI355X).

Every factor entry of two refactorizations is compared bit for bit with the
oracle's refactorization of the same matrices, and each solve meets the
backward-error bound eta <= 1e-12 on the host.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2306_14337_amd import binding, kktgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()
    yield


def test_full_size_factors_bitwise_and_eta():
    B, seed, steps = 70000, 103, 2
    print(f"case B={B} seed={seed} steps={steps} (library defaults)", flush=True)
    t0 = time.perf_counter()
    pat, seq = kktgen.make_sequence(B, seed, steps)
    print(f"  generated n={pat.n} nnz={len(pat.colind)} in {time.perf_counter() - t0:.1f} s",
          flush=True)
    s = binding.KKTSolver()
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    print(f"  analyzed, dense block {s.info().dense_tail}", flush=True)
    ora = oracle.OracleLU(pat.n, pat.rowptr, pat.colind, seq[0][0], tau=1e-10)
    f = ora.factors()
    n = pat.n
    rows = np.concatenate([f["Li"], f["Ui"]])
    cols = np.concatenate([np.repeat(np.arange(n), np.diff(f["Lp"])),
                           np.repeat(np.arange(n), np.diff(f["Up"]))])
    perm = np.lexsort((cols, rows))
    A_csr = None
    for k, (vals, b) in enumerate(seq):
        db = torch.from_numpy(b).to(DEV)
        s.refactor(torch.from_numpy(vals).to(DEV))
        x = s.solve(db).cpu().numpy()
        ora.refactor(vals)
        f = ora.factors()
        want = np.concatenate([f["Lx"], f["Ux"]])[perm]
        got = s.lu()[2]
        ndiff = int(np.sum(got.view(np.int64) != want.view(np.int64)))
        print(f"  step {k}: {len(want)} factor entries, {ndiff} differ", flush=True)
        assert ndiff == 0
        A_csr = pat.scipy(vals)
        e = np.abs(b - A_csr @ x).max() / (abs(A_csr).sum(1).max() * np.abs(x).max())
        print(f"  step {k}: eta {e:.3e}", flush=True)
        assert e <= 1e-12
