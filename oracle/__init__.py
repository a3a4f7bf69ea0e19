"""ctypes wrapper of the CPU FP64 oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

OK, WARN_SINGULAR, WARN_TINY_PIVOT, WARN_NOT_CONVERGED, WARN_PERTURBED = 0, 1, 2, 3, 4
ERR_ARG, ERR_STRUCT_SINGULAR = -1, -3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict IEEE: no contraction, explicit fma)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-mfma", "-fPIC", "-shared",
               "-Wall", "-Wno-unused-variable", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iters", C.c_int32), ("min_iters", C.c_int32),
                ("eta_target", C.c_double), ("method", C.c_int32)]


class _SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("eta", C.c_double),
                ("eta0", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.oracle_order_md.argtypes = [C.c_int32, P, P, P]
        L.oracle_order_md.restype = C.c_int
        L.oracle_match_scale.argtypes = [C.c_int32, P, P, P, P, P, P]
        L.oracle_match_scale.restype = C.c_int
        L.oracle_factor.argtypes = [C.c_int32, P, P, P, P, C.c_double, C.POINTER(C.c_int)]
        L.oracle_factor.restype = P
        L.oracle_lu_free.argtypes = [P]
        L.oracle_lu_sizes.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.oracle_lu_export.argtypes = [P] * 9
        L.oracle_lu_absprod.argtypes = [P, P, P]
        L.oracle_lu_growth.argtypes = [P]
        L.oracle_lu_growth.restype = C.c_double
        L.oracle_lu_apply_jacobi.argtypes = [P, P, C.c_int32, P]
        L.oracle_refactor.argtypes = [P, P, C.c_double]
        L.oracle_refactor.restype = C.c_int
        L.oracle_refactor_perturbed.argtypes = [P, P, C.c_double, C.c_double]
        L.oracle_refactor_perturbed.restype = C.c_int
        L.oracle_set_values.argtypes = [P, P]
        L.oracle_set_values.restype = C.c_int
        L.oracle_solve.argtypes = [P, C.c_char, C.c_int32, P, P, C.POINTER(_SolveOpts),
                                   C.POINTER(_SolveInfo)]
        L.oracle_solve.restype = C.c_int
        L.oracle_lu_apply.argtypes = [P, C.c_char, P, P]
        L.oracle_fgmres_trace.argtypes = [P, C.c_char, P, C.c_int32, P, P, P]
        L.oracle_fgmres_trace.restype = C.c_int
        L.oracle_grad.argtypes = [P, C.c_int32, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _csr(rowptr, colind):
    return (np.ascontiguousarray(rowptr, dtype=np.int64), np.ascontiguousarray(colind, dtype=np.int32))


def order_md(n: int, rowptr, colind) -> np.ndarray:
    """Exact minimum-degree ordering Q of pattern(A + A^T)."""
    rp, ci = _csr(rowptr, colind)
    Q = np.empty(n, dtype=np.int32)
    st = lib().oracle_order_md(n, _p(rp), _p(ci), _p(Q))
    if st != OK:
        raise ValueError(f"oracle_order_md failed ({st})")
    return Q


def match_scale(n: int, rowptr, colind, values):
    """Maximum-product matching and power-of-two scaling: (match, dr, dc) with
    match[j] = row matched to column j; raises if no perfect matching exists."""
    rp, ci = _csr(rowptr, colind)
    v = np.ascontiguousarray(values, dtype=np.float64)
    match = np.empty(n, dtype=np.int32)
    dr = np.empty(n, dtype=np.float64)
    dc = np.empty(n, dtype=np.float64)
    st = lib().oracle_match_scale(n, _p(rp), _p(ci), _p(v), _p(match), _p(dr), _p(dc))
    if st != OK:
        raise ValueError(f"oracle_match_scale failed ({st})")
    return match, dr, dc


def matched_scaled(n: int, rowptr, colind, values, match, dr, dc):
    """CSR of the matched and scaled matrix: row j is row match[j] of A with
    entries dr[match[j]] a_ij dc[c] (columns unchanged), and the position in
    A's values of each of its entries."""
    rp, ci = _csr(rowptr, colind)
    v = np.asarray(values, dtype=np.float64)
    nrp = np.zeros(n + 1, dtype=np.int64)
    cols, vals, src = [], [], []
    for j in range(n):
        i = int(match[j])
        lo, hi = int(rp[i]), int(rp[i + 1])
        cols.append(ci[lo:hi])
        vals.append(dr[i] * v[lo:hi] * dc[ci[lo:hi]])
        src.append(np.arange(lo, hi, dtype=np.int64))
        nrp[j + 1] = nrp[j] + (hi - lo)
    return (nrp, np.concatenate(cols).astype(np.int32), np.concatenate(vals),
            np.concatenate(src))


class OracleLU:
    """Pivoting LU of A' = Q^T A Q, refactorization and solves (plain CPU FP64)."""

    def __init__(self, n, rowptr, colind, values, Q=None, tau: float = 1.0):
        self.n = int(n)
        self.rowptr, self.colind = _csr(rowptr, colind)
        vals = np.ascontiguousarray(values, dtype=np.float64)
        if Q is None:
            Q = order_md(self.n, self.rowptr, self.colind)
        self.Q_in = np.ascontiguousarray(Q, dtype=np.int32)
        st = C.c_int(0)
        h = lib().oracle_factor(self.n, _p(self.rowptr), _p(self.colind), _p(vals), _p(self.Q_in),
                                float(tau), C.byref(st))
        self.status = st.value
        if not h:
            raise ValueError(f"oracle_factor failed (status {st.value})")
        self._h = C.c_void_p(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oracle_lu_free(h)
            self._h = None

    def sizes(self):
        a, b = C.c_int64(0), C.c_int64(0)
        lib().oracle_lu_sizes(self._h, C.byref(a), C.byref(b))
        return a.value, b.value

    def factors(self):
        """dict with P, Q and CSC L (strict) / U (diag last) in pivot order."""
        lnz, unz = self.sizes()
        n = self.n
        P = np.empty(n, np.int32)
        Q = np.empty(n, np.int32)
        Lp = np.empty(n + 1, np.int64)
        Li = np.empty(lnz, np.int32)
        Lx = np.empty(lnz, np.float64)
        Up = np.empty(n + 1, np.int64)
        Ui = np.empty(unz, np.int32)
        Ux = np.empty(unz, np.float64)
        lib().oracle_lu_export(self._h, _p(P), _p(Q), _p(Lp), _p(Li), _p(Lx), _p(Up), _p(Ui), _p(Ux))
        return dict(P=P, Q=Q, Lp=Lp, Li=Li, Lx=Lx, Up=Up, Ui=Ui, Ux=Ux)

    def absprod(self):
        lnz, unz = self.sizes()
        sL = np.empty(lnz, np.float64)
        sU = np.empty(unz, np.float64)
        lib().oracle_lu_absprod(self._h, _p(sL), _p(sU))
        return sL, sU

    def refactor(self, values, tiny_rel: float = 1e-18, perturb_rel: float = 0.0) -> int:
        """Refactorization; perturb_rel > 0 turns on static pivoting."""
        vals = np.ascontiguousarray(values, dtype=np.float64)
        if perturb_rel > 0.0:
            return lib().oracle_refactor_perturbed(self._h, _p(vals), float(tiny_rel),
                                                  float(perturb_rel))
        return lib().oracle_refactor(self._h, _p(vals), float(tiny_rel))

    def set_values(self, values) -> int:
        """Change the matrix seen by residuals but keep the (now stale) factors."""
        self._vals_keep = np.ascontiguousarray(values, dtype=np.float64)
        return lib().oracle_set_values(self._h, _p(self._vals_keep))

    def solve(self, b, op: str = "N", restart=20, max_iters=20, min_iters=0, eta_target=1e-12,
              method: str = "fgmres"):
        """method "fgmres" (FGMRES-CGS2) or "ir" (classical iterative refinement)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        nrhs = b.size // self.n
        x = np.empty_like(b)
        o = _SolveOpts(restart, max_iters, min_iters, eta_target, 1 if method == "ir" else 0)
        info = _SolveInfo()
        st = lib().oracle_solve(self._h, op.encode(), nrhs, _p(b), _p(x), C.byref(o), C.byref(info))
        return x, dict(status=st, iters=info.iters, converged=info.converged, eta=info.eta,
                       eta0=info.eta0)

    def apply(self, b, op: str = "N"):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty_like(b)
        lib().oracle_lu_apply(self._h, op.encode(), _p(b), _p(x))
        return x

    def apply_jacobi(self, b, sweeps: int):
        """Sweep-based approximate M^{-1} b (op 'N')."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty_like(b)
        lib().oracle_lu_apply_jacobi(self._h, _p(b), int(sweeps), _p(x))
        return x

    def growth(self) -> float:
        """max |u_ij| / ||A||_inf of the current factors."""
        return float(lib().oracle_lu_growth(self._h))

    def fgmres_trace(self, b, iters: int, prec: str = "L"):
        n = self.n
        b = np.ascontiguousarray(b, dtype=np.float64)
        V = np.zeros((iters + 1, n))
        Z = np.zeros((iters, n))
        H = np.zeros((iters, iters + 1))
        k = lib().oracle_fgmres_trace(self._h, prec.encode(), _p(b), iters, _p(V), _p(Z), _p(H))
        return k, V.T, Z.T, H.T

    def grad(self, lam, x):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        nrhs = lam.size // self.n
        g = np.empty(int(self.rowptr[-1]), np.float64)
        lib().oracle_grad(self._h, nrhs, _p(lam), _p(x), _p(g))
        return g


def csc_to_dense(n, p, i, x):
    D = np.zeros((n, n))
    for j in range(n):
        D[i[p[j]:p[j + 1]], j] = x[p[j]:p[j + 1]]
    return D
