"""Seeded synthetic ACOPF-shaped KKT systems (the only module shared by the
oracle side and the GPU side).

It draws random numbers and lays out sparsity patterns; it performs none of the
solver's arithmetic (no ordering, no factorization, no solve, no residual).

Why a synthetic generator: the paper evaluates on the ACTIVSg synthetic grids
(Section 3, Table "tab:descr") driven by ExaGO/HiOp, which are not available
here.  The systems produced below have the block form of the paper's KKT
matrix (Section 2, eq. "eq:kktlinear"), [[H + D_y, J], [J^T, 0]], written in
the equivalent symmetric arrangement

    K = [[W + Sigma, J^T],
         [J,        -1e-8 * I]]

where W plays H (a sparse symmetric Hessian whose coupling follows the grid's
lines), Sigma plays D_y (a positive diagonal spanning many orders of magnitude
as the barrier parameter shrinks), and the -1e-8 block is the interior
method's regularization that Section 5 relies on for pivot reuse.  All K_k of
a sequence share one pattern (Section 2, last paragraph); only Sigma changes
between steps, mimicking interior-point iterations.

Recipe (every choice the paper leaves open is a stated reading):
  1. B bus coordinates uniform in [0,1)^2.
  2. Candidate lines: the symmetrized 8-nearest-neighbour graph.
  3. Tree lines: Kruskal over the candidates in random order (a random
     spanning tree of the kNN graph, so the grid stays geographic); leftover
     components are joined by one link each.
  4. Extra lines: round(0.4 B) distinct candidates not in the tree.
  5. Generators: round(0.2 B) distinct buses.
  6. Primal variables [vm(B), va(B), pg(G), qg(G), s1(l), s2(l)];
     constraint rows [P(B), Q(B), F1(l), F2(l)]; n = 10 B - 4 when 0.4B and
     0.2B are integers.
  7. W pattern: a 2x2 (vm,va) block per bus, the 2x2 bus-bus coupling block of
     every line in both directions, and a diagonal for pg, qg, s1, s2.  The
     upper triangle (with the diagonal) is N(0,1), mirrored; then
     W_ii += sum_j |W_ij| (absolute row sum including the diagonal).
  8. Sigma = 10**U(-8, 8) on the primal variables.
  9. J: P_i touches vm/va of bus i and of its line neighbours plus pg_i if bus
     i has a generator; Q_i the same with qg_i; F1_l touches vm/va of both
     ends and s1_l; F2_l the same with s2_l.  Values N(0,1).
 10. Full CSR (both triangles), columns sorted, int64 row pointers, int32
     column indices, float64 values.
 11. Perturbed instances (scenario batches): N(0, 0.05) added to the raw W
     draws (before the diagonal shift, which is recomputed) and to J.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

REG = 1e-8  # magnitude of the (2,2) regularization block


@dataclasses.dataclass
class KKTPattern:
    """Pattern and fixed values of one synthetic KKT family.

    ``base_values`` holds K with Sigma = 0; ``values(sigma)`` adds Sigma on the
    primal diagonal positions ``sigma_pos``.
    """

    B: int
    n: int
    n_p: int
    m: int
    rowptr: np.ndarray  # int64 [n+1]
    colind: np.ndarray  # int32 [nnz]
    base_values: np.ndarray  # float64 [nnz]
    sigma_pos: np.ndarray  # int64 [n_p], position of K[i,i] for primal i
    seed: int

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def values(self, sigma: np.ndarray) -> np.ndarray:
        v = self.base_values.copy()
        v[self.sigma_pos] += sigma
        return v

    def scipy(self, values: np.ndarray) -> sp.csr_matrix:
        return sp.csr_matrix((values, self.colind, self.rowptr), shape=(self.n, self.n))


def draw_sigma(rng: np.random.Generator, n_p: int) -> np.ndarray:
    return 10.0 ** rng.uniform(-8.0, 8.0, size=n_p)


def _grid(B: int, rng: np.random.Generator):
    """Bus coordinates, line list (a<b pairs) and generator buses."""
    xy = rng.random((B, 2))
    k = min(9, B)
    _, nbr = cKDTree(xy).query(xy, k=k)
    nbr = np.asarray(nbr).reshape(B, k)
    a = np.repeat(np.arange(B), k - 1)
    b = nbr[:, 1:].reshape(-1)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    keep = lo != hi
    cand = np.unique(np.stack([lo[keep], hi[keep]], 1), axis=0)

    # Kruskal over the candidates in random order
    order = rng.permutation(len(cand))
    parent = np.arange(B)

    def find(x):
        root = x
        while parent[root] != root:
            root = parent[root]
        while parent[x] != root:
            parent[x], x = root, parent[x]
        return root

    in_tree = np.zeros(len(cand), dtype=bool)
    count = 0
    for e in order:
        u, v = cand[e]
        ru, rv = find(u), find(v)
        if ru != rv:
            parent[ru] = rv
            in_tree[e] = True
            count += 1
            if count == B - 1:
                break
    tree = cand[in_tree]
    # join leftover components, one link each (smallest bus of consecutive components)
    roots = np.array([find(x) for x in range(B)])
    comps = sorted({int(r) for r in roots}, key=lambda r: int(np.min(np.nonzero(roots == r)[0])))
    links = []
    for c0, c1 in zip(comps[:-1], comps[1:]):
        u = int(np.min(np.nonzero(roots == c0)[0]))
        v = int(np.min(np.nonzero(roots == c1)[0]))
        links.append((min(u, v), max(u, v)))
    if links:
        tree = np.concatenate([tree, np.array(links, dtype=tree.dtype)], 0)

    rest = cand[~in_tree]
    n_extra = min(int(round(0.4 * B)), len(rest))
    extra = rest[rng.choice(len(rest), size=n_extra, replace=False)] if n_extra else rest[:0]
    lines = np.concatenate([tree, extra], 0).astype(np.int64)
    n_gen = int(round(0.2 * B))
    gens = np.sort(rng.choice(B, size=n_gen, replace=False)).astype(np.int64)
    return lines, gens


@dataclasses.dataclass
class _Structure:
    B: int
    G: int
    L: int
    n_p: int
    m: int
    w_rows: np.ndarray  # upper-triangle W entries (row <= col)
    w_cols: np.ndarray
    j_rows: np.ndarray  # J entries (constraint row, primal column)
    j_cols: np.ndarray


def _structure(B: int, lines: np.ndarray, gens: np.ndarray) -> _Structure:
    G, L = len(gens), len(lines)
    vm = np.arange(B)
    va = B + np.arange(B)
    pg0, qg0 = 2 * B, 2 * B + G
    s10, s20 = 2 * B + 2 * G, 2 * B + 2 * G + L
    n_p = 2 * B + 2 * G + 2 * L
    m = 2 * B + 2 * L

    wr, wc = [], []
    # per-bus 2x2 block (upper triangle): (vm,vm) (vm,va) (va,va)
    wr += [vm, vm, va]
    wc += [vm, va, va]
    # per-line coupling blocks vm/va_a x vm/va_b; keep the upper-triangle copy
    a, b = lines[:, 0], lines[:, 1]
    for ra in (vm[a], va[a]):
        for cb in (vm[b], va[b]):
            wr.append(np.minimum(ra, cb))
            wc.append(np.maximum(ra, cb))
    diag = np.arange(2 * B, n_p)
    wr.append(diag)
    wc.append(diag)
    w_rows = np.concatenate(wr)
    w_cols = np.concatenate(wc)

    # J rows
    adj = [[] for _ in range(B)]
    for u, v in lines:
        adj[u].append(v)
        adj[v].append(u)
    jr, jc = [], []
    gen_idx = -np.ones(B, dtype=np.int64)
    gen_idx[gens] = np.arange(G)
    for i in range(B):
        buses = np.array(sorted([i] + adj[i]), dtype=np.int64)
        for q, g0 in ((0, pg0), (1, qg0)):
            row = q * B + i
            cols = np.concatenate([vm[buses], va[buses]])
            if gen_idx[i] >= 0:
                cols = np.append(cols, g0 + gen_idx[i])
            jr.append(np.full(len(cols), row))
            jc.append(cols)
    ln = np.arange(L)
    for q, s0 in ((0, s10), (1, s20)):
        row = 2 * B + q * L + ln
        for col in (vm[a], va[a], vm[b], va[b], s0 + ln):
            jr.append(row)
            jc.append(col)
    j_rows = np.concatenate(jr)
    j_cols = np.concatenate(jc)
    return _Structure(B, G, L, n_p, m, w_rows, w_cols, j_rows, j_cols)


def _assemble(st: _Structure, w_raw: np.ndarray, j_val: np.ndarray, seed: int) -> KKTPattern:
    n_p, m = st.n_p, st.m
    n = n_p + m
    off = st.w_rows != st.w_cols
    # symmetric W from the upper-triangle draws
    r = np.concatenate([st.w_rows, st.w_cols[off]])
    c = np.concatenate([st.w_cols, st.w_rows[off]])
    v = np.concatenate([w_raw, w_raw[off]])
    absrow = np.bincount(r, weights=np.abs(v), minlength=n_p)
    # diagonal shift W_ii += sum_j |W_ij|
    is_diag = r == c
    v = v.copy()
    v[is_diag] += absrow[r[is_diag]]
    rows = np.concatenate([r, st.j_cols, n_p + st.j_rows, n_p + np.arange(m)])
    cols = np.concatenate([c, n_p + st.j_rows, st.j_cols, n_p + np.arange(m)])
    vals = np.concatenate([v, j_val, j_val, np.full(m, -REG)])
    K = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    K.sort_indices()
    if K.nnz != len(vals):
        raise AssertionError("duplicate entries in the KKT pattern")
    rowptr = K.indptr.astype(np.int64)
    colind = K.indices.astype(np.int32)
    values = K.data.astype(np.float64)
    # positions of the primal diagonal
    sigma_pos = np.empty(n_p, dtype=np.int64)
    for_rows = np.arange(n_p)
    starts, ends = rowptr[:n_p], rowptr[1 : n_p + 1]
    for i in for_rows:
        seg = colind[starts[i] : ends[i]]
        sigma_pos[i] = starts[i] + int(np.searchsorted(seg, i))
    return KKTPattern(st.B, n, n_p, m, rowptr, colind, values, sigma_pos, seed)


def make_kkt(B: int, seed: int, perturb_seed: int | None = None, _cache={}) -> KKTPattern:
    """Synthetic KKT family for ``B`` buses (pattern + Sigma-free values).

    ``perturb_seed`` (scenario instances) adds N(0, 0.05) to the raw W and J
    draws of the base family drawn from ``seed``.
    """
    key = (B, seed)
    if key not in _cache:
        rng = np.random.default_rng(seed)
        lines, gens = _grid(B, rng)
        st = _structure(B, lines, gens)
        w_raw = rng.standard_normal(len(st.w_rows))
        j_val = rng.standard_normal(len(st.j_rows))
        _cache.clear()
        _cache[key] = (st, w_raw, j_val)
    st, w_raw, j_val = _cache[key]
    if perturb_seed is not None:
        prng = np.random.default_rng(perturb_seed)
        w_raw = w_raw + prng.normal(0.0, 0.05, size=len(w_raw))
        j_val = j_val + prng.normal(0.0, 0.05, size=len(j_val))
    return _assemble(st, w_raw, j_val, seed)


def make_sequence(B: int, seed: int, steps: int, nrhs: int = 1):
    """A same-pattern sequence: list of (values, rhs) with Sigma redrawn per step.

    Step k draws from ``default_rng(seed * 1000 + k)``: Sigma first, then the
    right-hand sides (column-major n x nrhs, flattened).
    """
    pat = make_kkt(B, seed)
    seq = []
    for k in range(steps):
        rng = np.random.default_rng(seed * 1000 + k)
        sigma = draw_sigma(rng, pat.n_p)
        rhs = rng.standard_normal(pat.n * nrhs)
        seq.append((pat.values(sigma), rhs))
    return pat, seq


def make_batch_group_a(B: int, seed: int, count: int):
    """Scenario group sharing one pattern: per-instance W/J perturbation and Sigma."""
    out = []
    for i in range(count):
        pat = make_kkt(B, seed, perturb_seed=seed * 1000 + i)
        rng = np.random.default_rng(seed * 100000 + i)
        sigma = draw_sigma(rng, pat.n_p)
        rhs = rng.standard_normal(pat.n)
        out.append((pat, pat.values(sigma), rhs))
    return out


def group_b_sizes(seed: int, count: int, lo: int = 500, hi: int = 5000) -> np.ndarray:
    return np.random.default_rng(seed).integers(lo, hi + 1, size=count)


def make_batch_group_b(seed: int, size_seed: int, count: int):
    """Uneven scenario group: instance i has its own B_i ~ U[500, 5000] pattern."""
    out = []
    for i, B in enumerate(group_b_sizes(size_seed, count)):
        pat = make_kkt(int(B), seed * 1000 + i)
        rng = np.random.default_rng(seed * 100000 + i)
        sigma = draw_sigma(rng, pat.n_p)
        rhs = rng.standard_normal(pat.n)
        out.append((pat, pat.values(sigma), rhs))
    return out


def random_sparse(n: int, density: float, seed: int, diag: bool = True, sym_pattern: bool = False):
    """Small random sparse test matrix (CSR arrays); values N(0,1)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    if sym_pattern:
        mask = mask | mask.T
    if diag:
        np.fill_diagonal(mask, True)
    vals = rng.standard_normal((n, n)) * mask
    # keep structural entries even where a draw is exactly zero
    r, c = np.nonzero(mask)
    v = vals[r, c]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, c.astype(np.int32), v.astype(np.float64)
