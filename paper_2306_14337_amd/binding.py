"""Thin ctypes binding of ``libkktlu.so`` (the C ABI in ``include/kkt_lu.h``).

Argument marshalling only: every step of analyze / refactor / solve runs in the
native library.  PyTorch supplies device memory (float64 CUDA tensors on
ROCm) and the current HIP stream.  There is no fallback: if the library is not
built, or no GPU is visible for the device calls, these functions raise.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libkktlu.so")

OK = 0
WARN_NUMERICALLY_SINGULAR = 1
WARN_TINY_PIVOT = 2
WARN_NOT_CONVERGED = 3
WARN_PERTURBED_PIVOT = 4
WARN_REANALYZED = 5
ERR_INVALID_ARG = -1
ERR_BAD_PATTERN = -2
ERR_STRUCTURALLY_SINGULAR = -3
ERR_STATE = -4
ERR_OUT_OF_MEMORY = -5
ERR_DEVICE = -6
ERR_NONFINITE = -7
ERR_TOO_LARGE = -8

EXPORTS = [
    "kkt_options_default", "kkt_create", "kkt_destroy", "kkt_analyze", "kkt_refactor",
    "kkt_update_matrix", "kkt_solve", "kkt_grad_values", "kkt_sync_report", "kkt_get_info", "kkt_get_perm",
    "kkt_get_lu", "kkt_last_error", "kkt_analysis_create", "kkt_analysis_info",
    "kkt_analysis_perm", "kkt_analysis_lu", "kkt_analysis_levels", "kkt_analysis_destroy",
    "kkt_analyze_batch", "kkt_batch_layout", "kkt_batch_eta", "kkt_graph_capture",
    "kkt_graph_launch", "kkt_reanalyze", "kkt_solve_noalloc", "kkt_get_scaling",
    "kkt_analysis_scaling", "kkt_debug_timeline", "kkt_analyze_shared",
]


class KKTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"kkt status {status}: {msg}")
        self.status = status


class Options(C.Structure):
    _fields_ = [("ordering", C.c_int32), ("pivot_tau", C.c_double), ("fgmres_restart", C.c_int32),
                ("fgmres_max_iters", C.c_int32), ("min_iters", C.c_int32),
                ("eta_target", C.c_double), ("tiny_pivot_rel", C.c_double), ("device", C.c_int32),
                ("schedule", C.c_int32), ("sync_mode", C.c_int32),
                ("solve_entries_per_lane", C.c_int32), ("refactor_waves_per_block", C.c_int32),
                ("solve_thin_rows", C.c_int32), ("dense_tail", C.c_int32),
                ("solve_blocks_per_cu", C.c_int32), ("solve_chain", C.c_int32),
                ("refactor_map", C.c_int32), ("refactor_crit_height", C.c_int32),
                ("refactor_waves_per_cu", C.c_int32), ("refine", C.c_int32),
                ("auto_reanalyze", C.c_int32), ("solve_jacobi_sweeps", C.c_int32),
                ("refactor_short_rows", C.c_int32), ("pivot_perturb_rel", C.c_double),
                ("refactor_long_rows", C.c_int32), ("refine_sync", C.c_int32),
                ("refine_budget", C.c_int32), ("dense_lu", C.c_int32),
                ("debug_spin_limit", C.c_int32), ("debug_schedule", C.c_int32),
                ("matching", C.c_int32), ("refactor_micro_rows", C.c_int32),
                ("debug_timeline", C.c_int32), ("refactor_short_band", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("warnings", C.c_int32), ("iters", C.c_int32), ("eta", C.c_double),
                ("eta0", C.c_double), ("min_pivot", C.c_double), ("max_pivot", C.c_double),
                ("anorm_inf", C.c_double), ("growth", C.c_double)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("nnz_l", C.c_int64), ("nnz_u", C.c_int64),
                ("levels", C.c_int32), ("levels_u", C.c_int32), ("analyze_status", C.c_int32),
                ("device_bytes", C.c_int64), ("analyze_seconds", C.c_double),
                ("dense_tail", C.c_int32), ("factor_epoch", C.c_int64),
                ("levels_sparse", C.c_int32), ("solve_block_levels", C.c_int32 * 2)]


_lib = None


def lib():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.kkt_options_default.argtypes = [C.POINTER(Options)]
        L.kkt_options_default.restype = None
        L.kkt_create.argtypes = [C.POINTER(Options), C.POINTER(P)]
        L.kkt_destroy.argtypes = [P]
        L.kkt_analyze.argtypes = [P, C.c_int32, C.c_int64, P, P, P, P]
        L.kkt_refactor.argtypes = [P, P, P]
        L.kkt_reanalyze.argtypes = [P, P, P]
        L.kkt_update_matrix.argtypes = [P, P, P]
        L.kkt_solve.argtypes = [P, C.c_char, C.c_int32, P, P, P]
        L.kkt_solve_noalloc.argtypes = [P, C.c_char, C.c_int32, P, P, P]
        L.kkt_grad_values.argtypes = [P, C.c_int32, P, P, P, P]
        L.kkt_sync_report.argtypes = [P, C.POINTER(Report)]
        L.kkt_get_info.argtypes = [P, C.POINTER(Info)]
        L.kkt_get_perm.argtypes = [P, P, P]
        L.kkt_get_scaling.argtypes = [P, P, P, P]
        L.kkt_debug_timeline.argtypes = [P, P]
        L.kkt_analysis_scaling.argtypes = [P, P, P, P]
        L.kkt_get_lu.argtypes = [P, P, P, P]
        L.kkt_last_error.argtypes = [P]
        L.kkt_last_error.restype = C.c_char_p
        L.kkt_analysis_create.argtypes = [C.POINTER(Options), C.c_int32, C.c_int64, P, P, P, P,
                                          C.POINTER(P), C.c_char_p, C.c_int32]
        L.kkt_analysis_info.argtypes = [P, C.POINTER(Info)]
        L.kkt_analysis_perm.argtypes = [P, P, P]
        L.kkt_analysis_lu.argtypes = [P, P, P, P]
        L.kkt_analysis_levels.argtypes = [P, P, P]
        L.kkt_analysis_destroy.argtypes = [P]
        L.kkt_analysis_destroy.restype = None
        L.kkt_analyze_batch.argtypes = [P, C.c_int32, P, P, P, P, P, C.c_int32, P]
        L.kkt_analyze_shared.argtypes = [P, C.c_int32, C.c_int64, P, P, P, C.c_int32]
        L.kkt_batch_layout.argtypes = [P, P, P]
        L.kkt_batch_eta.argtypes = [P, P]
        L.kkt_graph_capture.argtypes = [P, P, P, P, P]
        L.kkt_graph_launch.argtypes = [P, P]
        _lib = L
    return _lib


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def options(**kw) -> Options:
    o = Options()
    lib().kkt_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _csr_host(rowptr, colind, values):
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(colind, dtype=np.int32)
    v = np.ascontiguousarray(values, dtype=np.float64)
    return rp, ci, v


class HostAnalysis:
    """The analysis phase alone, on the host (``kkt_analysis_*``)."""

    def __init__(self, n, rowptr, colind, values0, user_q=None, **opts):
        rp, ci, v = _csr_host(rowptr, colind, values0)
        q = None if user_q is None else np.ascontiguousarray(user_q, dtype=np.int32)
        o = options(**opts)
        h = C.c_void_p()
        msg = C.create_string_buffer(512)
        st = lib().kkt_analysis_create(C.byref(o), int(n), int(rp[-1]), _np_ptr(rp), _np_ptr(ci),
                                       _np_ptr(v), None if q is None else _np_ptr(q), C.byref(h),
                                       msg, 512)
        if st < 0:
            raise KKTError(st, msg.value.decode())
        self.status = st
        self._h = h
        self.n = int(n)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.kkt_analysis_destroy(self._h)
            self._h = None

    def info(self) -> Info:
        i = Info()
        lib().kkt_analysis_info(self._h, C.byref(i))
        return i

    def perm(self):
        P = np.empty(self.n, np.int32)
        Q = np.empty(self.n, np.int32)
        lib().kkt_analysis_perm(self._h, _np_ptr(P), _np_ptr(Q))
        return P, Q

    def lu(self):
        i = self.info()
        f = i.nnz_l + i.nnz_u
        rp = np.empty(self.n + 1, np.int64)
        ci = np.empty(f, np.int32)
        v = np.empty(f, np.float64)
        lib().kkt_analysis_lu(self._h, _np_ptr(rp), _np_ptr(ci), _np_ptr(v))
        return rp, ci, v

    def scaling(self):
        """(match, dr, dc) of an analysis with matching=1."""
        m = np.empty(self.n, np.int32)
        dr = np.empty(self.n, np.float64)
        dc = np.empty(self.n, np.float64)
        st = lib().kkt_analysis_scaling(self._h, _np_ptr(m), _np_ptr(dr), _np_ptr(dc))
        if st < 0:
            raise KKTError(st, "no matching in this analysis")
        return m, dr, dc

    def levels(self):
        i = self.info()
        lp = np.empty(i.levels + 1, np.int32)
        rows = np.empty(self.n, np.int32)
        lib().kkt_analysis_levels(self._h, _np_ptr(lp), _np_ptr(rows))
        return lp, rows


def _torch():
    import torch

    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_f64(t, n_expected=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n_expected is not None and t.numel() != n_expected:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n_expected}")
    return C.c_void_p(t.data_ptr())


@dataclasses.dataclass
class SolveReport:
    warnings: int
    iters: int
    eta: float
    eta0: float
    min_pivot: float
    max_pivot: float
    anorm_inf: float
    growth: float


class KKTSolver:
    """analyze(pattern + first values) once; refactor(values) and solve(rhs)
    per system of the sequence, all on one GPU."""

    def __init__(self, device: int = 0, **opts):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("KKTSolver needs a HIP GPU (no CPU fallback exists)")
        self.device = device
        o = options(device=device, **opts)
        h = C.c_void_p()
        st = lib().kkt_create(C.byref(o), C.byref(h))
        if st != OK:
            raise KKTError(st, "kkt_create failed")
        self._h = h
        self.options = o  # the options the handle was created with
        self.n = None
        self.nnz = None
        self.last_status = OK

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.kkt_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, st):
        self.last_status = st
        if st < 0:
            raise KKTError(st, lib().kkt_last_error(self._h).decode())
        return st

    def analyze(self, n, rowptr, colind, values0, user_q=None) -> int:
        rp, ci, v = _csr_host(rowptr, colind, values0)
        q = None if user_q is None else np.ascontiguousarray(user_q, dtype=np.int32)
        st = lib().kkt_analyze(self._h, int(n), int(rp[-1]), _np_ptr(rp), _np_ptr(ci), _np_ptr(v),
                               None if q is None else _np_ptr(q))
        self._check(st)
        self.n = int(n)
        self.nnz = int(rp[-1])
        return st

    def analyze_batch(self, patterns, inst_pattern) -> int:
        """Block-diagonal batch: patterns = [(n, rowptr, colind, values0), ...],
        inst_pattern[t] = pattern of instance t."""
        npat = len(patterns)
        keep = [_csr_host(rp, ci, v) for (_, rp, ci, v) in patterns]
        ns = np.array([int(p[0]) for p in patterns], np.int32)
        nnzs = np.array([int(k[0][-1]) for k in keep], np.int64)
        PP = C.c_void_p * npat
        rps = PP(*[k[0].ctypes.data for k in keep])
        cis = PP(*[k[1].ctypes.data for k in keep])
        vs = PP(*[k[2].ctypes.data for k in keep])
        ip = np.ascontiguousarray(inst_pattern, dtype=np.int32)
        st = lib().kkt_analyze_batch(self._h, npat, _np_ptr(ns), _np_ptr(nnzs), rps, cis, vs,
                                     len(ip), _np_ptr(ip))
        self._check(st)
        self.count = len(ip)
        ro = np.empty(self.count + 1, np.int64)
        no = np.empty(self.count + 1, np.int64)
        self._check(lib().kkt_batch_layout(self._h, _np_ptr(ro), _np_ptr(no)))
        self.row_offset, self.nnz_offset = ro, no
        self.n = int(ro[-1])
        self.nnz = int(no[-1])
        return st

    def analyze_shared(self, n, rowptr, colind, values0, count) -> int:
        """count instances of one pattern sharing one analysis and one copy of
        every index structure (values and vectors per instance, back to
        back; the handle then answers as a block-diagonal batch)."""
        rp, ci, v = _csr_host(rowptr, colind, values0)
        st = lib().kkt_analyze_shared(self._h, int(n), int(rp[-1]), _np_ptr(rp), _np_ptr(ci),
                                      _np_ptr(v), int(count))
        self._check(st)
        self.count = int(count)
        ro = np.empty(self.count + 1, np.int64)
        no = np.empty(self.count + 1, np.int64)
        self._check(lib().kkt_batch_layout(self._h, _np_ptr(ro), _np_ptr(no)))
        self.row_offset, self.nnz_offset = ro, no
        self.n = int(ro[-1])
        self.nnz = int(no[-1])
        return st

    def batch_eta(self) -> np.ndarray:
        e = np.empty(self.count, np.float64)
        self._check(lib().kkt_batch_eta(self._h, _np_ptr(e)))
        return e

    def graph_capture(self, values, b, x, stream) -> int:
        """Capture refactor + direct solve + residual check on a non-default stream."""
        st = lib().kkt_graph_capture(self._h, _dev_f64(values, self.nnz, "values"),
                                     _dev_f64(b, name="b"), _dev_f64(x, b.numel(), "x"),
                                     C.c_void_p(stream.cuda_stream))
        self._graph_keep = (values, b, x)
        return self._check(st)

    def graph_launch(self, stream) -> int:
        return self._check(lib().kkt_graph_launch(self._h, C.c_void_p(stream.cuda_stream)))

    def refactor(self, values, stream=None) -> int:
        p = _dev_f64(values, self.nnz, "values")
        return self._check(lib().kkt_refactor(self._h, p, _stream_ptr(stream)))

    def reanalyze(self, values, stream=None) -> int:
        """Re-run the pivoting pass on new values (keeps the ordering); its
        factors become the current factors."""
        p = _dev_f64(values, self.nnz, "values")
        return self._check(lib().kkt_reanalyze(self._h, p, _stream_ptr(stream)))

    def update_matrix(self, values, stream=None) -> int:
        """New matrix for the residuals; the current factors stay as preconditioner."""
        p = _dev_f64(values, self.nnz, "values")
        return self._check(lib().kkt_update_matrix(self._h, p, _stream_ptr(stream)))

    def solve(self, b, x=None, op: str = "N", stream=None):
        torch = _torch()
        if b.numel() % self.n:
            raise ValueError("b must hold n * nrhs entries")
        nrhs = b.numel() // self.n
        if x is None:
            x = torch.empty_like(b)
        st = lib().kkt_solve(self._h, op.encode(), nrhs, _dev_f64(b, name="b"),
                             _dev_f64(x, b.numel(), "x"), _stream_ptr(stream))
        self._check(st)
        return x

    def solve_noalloc(self, b, x, op: str = "N", stream=None):
        """kkt_solve_noalloc: the solve with its per-call scratch in the
        library's static device array (no allocation; x must be given)."""
        if b.numel() % self.n:
            raise ValueError("b must hold n * nrhs entries")
        nrhs = b.numel() // self.n
        st = lib().kkt_solve_noalloc(self._h, op.encode(), nrhs, _dev_f64(b, name="b"),
                                     _dev_f64(x, b.numel(), "x"), _stream_ptr(stream))
        self._check(st)
        return x

    def grad_values(self, lam, x, out=None, stream=None):
        torch = _torch()
        nrhs = lam.numel() // self.n
        if out is None:
            out = torch.empty(self.nnz, dtype=torch.float64, device=lam.device)
        st = lib().kkt_grad_values(self._h, nrhs, _dev_f64(lam, name="lambda"),
                                   _dev_f64(x, lam.numel(), "x"), _dev_f64(out, self.nnz, "grad"),
                                   _stream_ptr(stream))
        self._check(st)
        return out

    def report(self) -> SolveReport:
        r = Report()
        self._check(lib().kkt_sync_report(self._h, C.byref(r)))
        return SolveReport(r.warnings, r.iters, r.eta, r.eta0, r.min_pivot, r.max_pivot,
                           r.anorm_inf, r.growth)

    def info(self) -> Info:
        i = Info()
        self._check(lib().kkt_get_info(self._h, C.byref(i)))
        return i

    def factor_epoch(self) -> int:
        """Counter of the calls that replaced the factors or the matrix."""
        return int(self.info().factor_epoch)

    def perm(self):
        P = np.empty(self.n, np.int32)
        Q = np.empty(self.n, np.int32)
        self._check(lib().kkt_get_perm(self._h, _np_ptr(P), _np_ptr(Q)))
        return P, Q

    def scaling(self):
        """(match, dr, dc) of an analysis with matching=1."""
        m = np.empty(self.n, np.int32)
        dr = np.empty(self.n, np.float64)
        dc = np.empty(self.n, np.float64)
        self._check(lib().kkt_get_scaling(self._h, _np_ptr(m), _np_ptr(dr), _np_ptr(dc)))
        return m, dr, dc

    def debug_timeline(self) -> np.ndarray:
        """Row timeline of the last refactorization (handle created with
        debug_timeline=1): n x 4 int64 (start, last poll that found an input
        missing, end in ns; kernel kind 1 micro / 2 list / 3 long-row; -1 and
        0 for rows outside the two band kernels)."""
        out = np.empty((self.n, 4), np.int64)
        self._check(lib().kkt_debug_timeline(self._h, _np_ptr(out)))
        return out

    def lu(self, values: bool = True):
        i = self.info()
        f = i.nnz_l + i.nnz_u
        rp = np.empty(self.n + 1, np.int64)
        ci = np.empty(f, np.int32)
        v = np.empty(f, np.float64) if values else None
        self._check(lib().kkt_get_lu(self._h, _np_ptr(rp), _np_ptr(ci),
                                     None if v is None else _np_ptr(v)))
        return rp, ci, v


class KKTSolveFn:
    """Differentiable x = A(values)^{-1} b on a fixed pattern.

    ``KKTSolveFn.apply(solver, values, b)`` refactorizes with ``values`` and
    solves; the backward pass solves A^T lambda = dL/dx with the same factors
    (transposed) and returns dL/db = lambda and dL/dvalues[p] =
    -sum_r lambda_r[i] x_r[j] for every stored entry p = (i, j) of the pattern.
    b is n (one right-hand side) or n * nrhs (column-major).  backward raises
    if the solver's factors were replaced after the forward pass (its factor
    epoch moved on), since the saved solution then belongs to other factors.
    """

    _fn = None

    @classmethod
    def apply(cls, solver: "KKTSolver", values, b):
        if cls._fn is None:
            torch = _torch()

            class _Fn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, solver, values, b):
                    solver.refactor(values.detach().contiguous())
                    x = solver.solve(b.detach().contiguous())
                    ctx.solver = solver
                    ctx.epoch = solver.factor_epoch()
                    ctx.save_for_backward(x)
                    return x

                @staticmethod
                def backward(ctx, gx):
                    (x,) = ctx.saved_tensors
                    s = ctx.solver
                    if s.factor_epoch() != ctx.epoch:
                        raise RuntimeError(
                            "KKTSolveFn.backward: the solver was refactorized after this forward "
                            "pass; its factors no longer belong to the saved solution (use one "
                            "solver per differentiated solve, or run backward first)")
                    lam = s.solve(gx.contiguous(), op="T")
                    gvals = s.grad_values(lam, x) if ctx.needs_input_grad[1] else None
                    gb = lam if ctx.needs_input_grad[2] else None
                    return None, gvals, gb

            cls._fn = _Fn
        return cls._fn.apply(solver, values, b)
