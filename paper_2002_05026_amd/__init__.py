"""Python binding of libd3m: the D3M dual block-LDL^T factorization and solve
on AMD MI355X (gfx950).

Argument marshalling only: every step of the factorization and solve runs in
the library's HIP kernels.  PyTorch provides device memory (the workspace,
K, B, X) and the current stream.  The library must be built (build.py); on
a machine without it the import of the native library fails loudly.

Sec. II of the paper (Moshfegh, Makris, Vouvakis 2019) defines the step:
the reduced matrix K is block-wise sparse with dense blocks coupling domain
interfaces, and the dual factorization/solution runs per nonzero block a
dense factorization, dense triangular solves and dense updates.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libd3m.so")

C128 = 0
C64_IR = 1
STATIC_WS_BYTES = 64 << 20  # D3M_STATIC_WS_BYTES of include/d3m.h

STATUS = {0: "ok", -1: "invalid argument", -2: "invalid block pattern or order", -3: "workspace too small",
          -4: "call out of sequence", -5: "HIP runtime error", -6: "watchdog (hang)", -7: "no device",
          1: "zero pivot", 2: "non-finite", 3: "refinement did not converge"}


class D3MError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {STATUS.get(code, code)} ({code})")
        self.code = code


class AnalyzeOptions(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("nworkers", ctypes.c_int32), ("sched", ctypes.c_int32),
                ("nelim", ctypes.c_int32), ("solve_tile", ctypes.c_int32), ("merge", ctypes.c_int32),
                ("rhs_groups", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("ir_host_sync", ctypes.c_int32),
                ("growth_dmin", ctypes.c_double), ("growth_lmax", ctypes.c_double),
                ("fallback", ctypes.c_int32), ("timing", ctypes.c_int32), ("dk_stored", ctypes.c_int32),
                ("pivot", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "N", "nblk", "npair", "k_len", "fill_blocks", "L_blocks", "nnz_L", "nnz_K", "etree_height", "max_S",
        "ntask_factor", "ntask_solve", "ntiles")] + [(k, ctypes.c_double) for k in (
            "flops_diag", "flops_trsm", "flops_update", "flops_factor", "solve_flops_per_rhs", "sim_factor_us")]


class RunInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("ir_iters", ctypes.c_int32), ("pivot_row", ctypes.c_int64),
                ("eta", ctypes.c_double), ("eta_hist", ctypes.c_double * 32), ("fallbacks", ctypes.c_int32),
                ("hang", ctypes.c_int32), ("t_factor_dag_ms", ctypes.c_double), ("t_solve_dag_ms", ctypes.c_double),
                ("n_factor_dag", ctypes.c_int32), ("n_solve_dag", ctypes.c_int32), ("knorm", ctypes.c_double)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes); every entry point of include/d3m.h
SIGNATURES = {
    "d3m_analyze": (_i32, [_i32, _i32p, _i64, _i32p, _i32p, _i32p, ctypes.POINTER(AnalyzeOptions),
                           ctypes.POINTER(_vp)]),
    "d3m_plan_query": (_i32, [_vp, ctypes.POINTER(PlanInfo)]),
    "d3m_plan_order": (_i32, [_vp, _i32p]),
    "d3m_plan_k_offsets": (_i32, [_vp, _i64p]),
    "d3m_plan_struct": (_i32, [_vp, _i32, _i32p, _i32p]),
    "d3m_plan_check": (_i32, [_vp, _i64p]),
    "d3m_plan_destroy": (None, [_vp]),
    "d3m_workspace_bytes": (_i32, [_vp, _i32, _i32, ctypes.POINTER(ctypes.c_size_t)]),
    "d3m_factor_bind": (_i32, [_vp, _i32, _vp, ctypes.c_size_t, _i32, ctypes.POINTER(Options),
                               ctypes.POINTER(_vp)]),
    "d3m_factor_bind_static": (_i32, [_vp, _i32, _i32, ctypes.POINTER(Options), ctypes.POINTER(_vp)]),
    "d3m_factorize": (_i32, [_vp, _vp, _vp]),
    "d3m_solve": (_i32, [_vp, _vp, _vp, _vp, _i32, _i64, _vp]),
    "d3m_adjoint": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _i64, _vp]),
    "d3m_reduce": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _i64, _i32, _vp]),
    "d3m_recover": (_i32, [_vp, _vp, _i64, _vp, _i64, _i32, _vp, _i64, _i32, _vp, _vp]),
    "d3m_status_sync": (_i32, [_vp, ctypes.POINTER(RunInfo)]),
    "d3m_factor_block": (_i32, [_vp, _i32, _i32, _vp]),
    "d3m_factor_destroy": (None, [_vp]),
    "d3m_factor_pivots": (_i32, [_vp, _i32, _i32p, _vp]),
    "d3m_factor_set_trace": (_i32, [_vp, _vp, ctypes.c_size_t]),
    "d3m_factor_tasks": (_i32, [_vp, _i32, _i32p, _i32p, _i32p, _i32p]),
    "d3m_batch_workspace_bytes": (_i32, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_size_t)]),
    "d3m_batch_create": (_i32, [_i32, ctypes.POINTER(_vp), _vp, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    "d3m_batch_run": (_i32, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i32p, _i64p,
                             _vp]),
    "d3m_batch_destroy": (None, [_vp]),
    "d3m_tune_gemm": (_i32, [_i32, _vp, ctypes.c_size_t, _i32p, ctypes.POINTER(ctypes.c_double), _i32p]),
    "d3m_debug_gemm": (_i32, [_i32, _i32, _i32, _i32, _i32, _i32, _vp, _i64, _vp, _vp, _i64, _vp, _i64,
                              ctypes.c_double, ctypes.c_double, _vp]),
    "d3m_status_string": (ctypes.c_char_p, [_i32]),
    "d3m_device_ok": (_i32, []),
}

_LIB = None


def lib():
    """The loaded libd3m (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libd3m.so not built ({LIB_PATH}); run paper_2002_05026_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _check(code: int, where: str):
    if code < 0:
        raise D3MError(code, where)
    return code


def _arr32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _p32(a):
    return a.ctypes.data_as(_i32p)


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Symbolic analysis: elimination order, block fill, tile DAGs (host only)."""

    def __init__(self, sizes, pairs, order=None, grid=None, tile: int = 0, nworkers: int = 0,
                 sched: int = 0, nelim: int = 0, solve_tile: int = 0, merge: int = 0, rhs_groups: int = 0):
        self.sizes = _arr32(sizes)
        self.pairs = _arr32(np.asarray(pairs).reshape(-1, 2))
        o = None if order is None else _arr32(order)
        g = None if grid is None else _arr32(grid)
        self.nelim = int(nelim)
        opts = AnalyzeOptions(int(tile), int(nworkers), int(sched), self.nelim, int(solve_tile), int(merge),
                              int(rhs_groups), 0)
        h = _vp()
        _check(lib().d3m_analyze(self.sizes.shape[0], _p32(self.sizes), self.pairs.shape[0], _p32(self.pairs),
                                 _p32(o) if o is not None else None, _p32(g) if g is not None else None,
                                 ctypes.byref(opts), ctypes.byref(h)), "d3m_analyze")
        self._h = h
        inf = PlanInfo()
        _check(lib().d3m_plan_query(self._h, ctypes.byref(inf)), "d3m_plan_query")
        self.info = {k: getattr(inf, k) for k, _ in PlanInfo._fields_}
        self.N = int(inf.N)
        self.nb = int(inf.nblk)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and h.value and _LIB is not None:
            _LIB.d3m_plan_destroy(h)
            self._h = None

    def order(self) -> np.ndarray:
        out = np.zeros(self.nb, dtype=np.int32)
        _check(lib().d3m_plan_order(self._h, _p32(out)), "d3m_plan_order")
        return out

    def k_offsets(self) -> np.ndarray:
        out = np.zeros(self.nb + self.pairs.shape[0] + 1, dtype=np.int64)
        _check(lib().d3m_plan_k_offsets(self._h, out.ctypes.data_as(_i64p)), "d3m_plan_k_offsets")
        return out

    def struct(self, I: int) -> list:
        out = np.zeros(self.nb, dtype=np.int32)
        cnt = _i32()
        _check(lib().d3m_plan_struct(self._h, int(I), _p32(out), ctypes.byref(cnt)), "d3m_plan_struct")
        return out[:cnt.value].tolist()

    def check(self) -> int:
        v = _i64()
        _check(lib().d3m_plan_check(self._h, ctypes.byref(v)), "d3m_plan_check")
        return int(v.value)

    def workspace_bytes(self, precision: int, nrhs_max: int) -> int:
        b = ctypes.c_size_t()
        _check(lib().d3m_workspace_bytes(self._h, int(precision), int(nrhs_max), ctypes.byref(b)),
               "d3m_workspace_bytes")
        return int(b.value)

    def factor(self, K, precision: int = C128, nrhs_max: int = 1, stream=None, **opts) -> "Factor":
        f = Factor(self, precision, nrhs_max, **opts)
        f.factorize(K, stream)
        return f


class Factor:
    """A numeric factor bound to a torch-owned device workspace, or with
    static_ws=True to the library's own static device array (no allocation;
    at most STATIC_WS_BYTES, one such factor per device at a time)."""

    def __init__(self, plan: Plan, precision: int = C128, nrhs_max: int = 1, tol: float = 1e-10,
                 max_iter: int = 10, ir_host_sync: bool = False, timing: bool = False, growth_dmin: float = 0.0,
                 growth_lmax: float = 0.0, fallback: bool = True, dk_stored: bool = False, device=None,
                 static_ws: bool = False, pivot: bool = False):
        import torch
        self.plan = plan
        self.precision = int(precision)
        self.nrhs_max = int(nrhs_max)
        opts = Options(float(tol), int(max_iter), int(bool(ir_host_sync)), float(growth_dmin), float(growth_lmax),
                       0 if fallback else -1, int(bool(timing)), int(bool(dk_stored)), int(bool(pivot)))
        h = _vp()
        if static_ws:
            self.ws = None
            _check(lib().d3m_factor_bind_static(plan._h, self.precision, self.nrhs_max, ctypes.byref(opts),
                                                ctypes.byref(h)), "d3m_factor_bind_static")
        else:
            nbytes = plan.workspace_bytes(precision, nrhs_max)
            dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
            base = self.ws.data_ptr()
            self._off = (-base) % 256
            _check(lib().d3m_factor_bind(plan._h, self.precision, ctypes.c_void_p(base + self._off), nbytes,
                                         self.nrhs_max, ctypes.byref(opts), ctypes.byref(h)), "d3m_factor_bind")
        self._h = h
        self.K = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and h.value and _LIB is not None:
            _LIB.d3m_factor_destroy(h)
            self._h = None

    def _checkK(self, K):
        import torch
        if K.dtype != torch.complex128 or not K.is_cuda or not K.is_contiguous():
            raise ValueError("K must be a contiguous complex128 CUDA tensor")
        if K.numel() != self.plan.info["k_len"]:
            raise ValueError(f"K has {K.numel()} elements, the plan needs {self.plan.info['k_len']}")

    def _checkB(self, B):
        import torch
        if B.dtype != torch.complex128 or not B.is_cuda or B.dim() != 2 or B.shape[1] != self.plan.N:
            raise ValueError("B must be a complex128 CUDA tensor of shape (nrhs, N)")
        if B.stride(1) != 1:
            raise ValueError("each right-hand side must be contiguous")
        if B.shape[0] > self.nrhs_max:
            raise ValueError(f"{B.shape[0]} right-hand sides exceed nrhs_max={self.nrhs_max}")

    def factorize(self, K, stream=None):
        self._checkK(K)
        self.K = K
        _check(lib().d3m_factorize(self._h, _ptr(K), _stream(stream)), "d3m_factorize")
        return self

    def solve(self, B, X=None, stream=None):
        """X = K^{-1} B; B is (nrhs, N) complex128 (each RHS a row)."""
        import torch
        if self.K is None:
            raise RuntimeError("factorize first")
        self._checkB(B)
        if X is None:
            X = torch.empty_like(B)
        _check(lib().d3m_solve(self._h, _ptr(self.K), _ptr(B), _ptr(X), B.shape[0], B.stride(0),
                               _stream(stream)), "d3m_solve")
        return X

    def adjoint(self, X, G, Lam=None, dK=None, want_dK: bool = True, stream=None):
        """Lambda = K^{-1} G and dK = -sym(Lambda X^T) on K's pattern (holomorphic)."""
        import torch
        self._checkB(G)
        if Lam is None:
            Lam = torch.empty_like(G)
        if want_dK and dK is None:
            dK = torch.empty_like(self.K)
        _check(lib().d3m_adjoint(self._h, _ptr(self.K), _ptr(X), _ptr(G), _ptr(Lam),
                                 _ptr(dK) if want_dK else None, G.shape[0], G.stride(0), _stream(stream)),
               "d3m_adjoint")
        return Lam, dK

    def reduce(self, A, F=None, stream=None):
        """Primal reduction with a partial-elimination plan: returns (Kred,
        Gred), the Schur complement on the blocks left (K layout of those
        blocks and the leading pairs) and, given F (nrhs, N), the reduced
        right-hand sides (nrhs, N_left)."""
        import torch
        self._checkK(A)
        nred = self.plan.nb - self.plan.nelim
        rows = int(self.plan.sizes[:nred].astype(np.int64).sum())
        npr = 0
        while npr < self.plan.pairs.shape[0] and self.plan.pairs[npr].max() < nred:
            npr += 1
        klen = int((self.plan.sizes[:nred].astype(np.int64) ** 2).sum() +
                   sum(int(self.plan.sizes[a]) * int(self.plan.sizes[b]) for a, b in self.plan.pairs[:npr].tolist()))
        Kred = torch.empty(klen, dtype=torch.complex128, device=A.device)
        G = None
        if F is not None:
            self._checkB(F)
            G = torch.empty((F.shape[0], rows), dtype=torch.complex128, device=A.device)
        self.K = A
        _check(lib().d3m_reduce(self._h, _ptr(A), _ptr(F) if F is not None else None,
                                F.stride(0) if F is not None else 0, _ptr(Kred),
                                _ptr(G) if G is not None else None, G.stride(0) if G is not None else 0,
                                F.shape[0] if F is not None else 1, _stream(stream)), "d3m_reduce")
        return Kred, G

    def recover(self, Xred, M=None, stream=None):
        """Primal recovery after reduce(A, F): the full primal solution U
        (nrhs, N) and, with port modes M (nports, N), S (nports, nrhs)."""
        import torch
        nr = Xred.shape[0]
        U = torch.empty((nr, self.plan.N), dtype=torch.complex128, device=Xred.device)
        S = None
        npt = 0
        if M is not None:
            npt = M.shape[0]
            S = torch.empty((nr, npt), dtype=torch.complex128, device=Xred.device)  # column-major nports x nrhs
        _check(lib().d3m_recover(self._h, _ptr(Xred), Xred.stride(0), _ptr(U), U.stride(0), nr,
                                 _ptr(M) if M is not None else None, M.stride(0) if M is not None else 0, npt,
                                 _ptr(S) if S is not None else None, _stream(stream)), "d3m_recover")
        return (U, S.t()) if M is not None else U

    def status(self) -> dict:
        ri = RunInfo()
        code = lib().d3m_status_sync(self._h, ctypes.byref(ri))
        hist = [v for v in ri.eta_hist if v >= 0]
        return {"status": int(code), "ir_iters": int(ri.ir_iters), "pivot_row": int(ri.pivot_row),
                "eta": float(ri.eta), "eta_hist": hist, "fallbacks": int(ri.fallbacks), "hang": int(ri.hang),
                "t_factor_dag_ms": float(ri.t_factor_dag_ms), "t_solve_dag_ms": float(ri.t_solve_dag_ms),
                "n_factor_dag": int(ri.n_factor_dag), "n_solve_dag": int(ri.n_solve_dag), "knorm": float(ri.knorm)}

    def set_trace(self, buf=None):
        """Record per-task timestamps of later DAG launches into the CUDA
        tensor buf (any dtype; its size in bytes is what counts; None stops)."""
        if buf is None:
            _check(lib().d3m_factor_set_trace(self._h, None, 0), "d3m_factor_set_trace")
        else:
            _check(lib().d3m_factor_set_trace(self._h, _ptr(buf), buf.numel() * buf.element_size()),
                   "d3m_factor_set_trace")
        self._trace = buf

    def tasks(self, solve: bool = False) -> dict:
        cnt = _i32()
        _check(lib().d3m_factor_tasks(self._h, int(solve), None, None, None, ctypes.byref(cnt)), "d3m_factor_tasks")
        n = cnt.value
        kinds = np.zeros(n, dtype=np.int32)
        panels = np.zeros(n, dtype=np.int32)
        mnk = np.zeros(3 * n, dtype=np.int32)
        _check(lib().d3m_factor_tasks(self._h, int(solve), _p32(kinds), _p32(panels), _p32(mnk), ctypes.byref(cnt)),
               "d3m_factor_tasks")
        return {"kind": kinds, "panel": panels, "mnk": mnk.reshape(n, 3)}

    def pivots(self, I: int):
        """(perm, doff) of user interface I of a pivoted factor (see d3m_factor_pivots)."""
        n = int(self.plan.sizes[I])
        perm = np.zeros(n, dtype=np.int32)
        doff = np.zeros(n, dtype=np.complex128)
        _check(lib().d3m_factor_pivots(self._h, int(I), _p32(perm), ctypes.c_void_p(doff.ctypes.data)),
               "d3m_factor_pivots")
        return perm, doff

    def block(self, J: int, I: int) -> np.ndarray:
        nJ, nI = int(self.plan.sizes[J]), int(self.plan.sizes[I])
        out = np.zeros(nJ * nI, dtype=np.complex128)
        _check(lib().d3m_factor_block(self._h, int(J), int(I), ctypes.c_void_p(out.ctypes.data)),
               "d3m_factor_block")
        return out.reshape(nJ, nI, order="F")


def debug_gemm(A, B, C, m, n, k, amode=0, i0=0, d=None, alpha=1.0, beta=0.0, lda=None, ldb=None, ldc=None,
               stream=None):
    """One tile product of the MFMA engine (see d3m_debug_gemm); tensors are
    1-D complex CUDA tensors holding the column-major operands."""
    import torch
    prec = C128 if C.dtype == torch.complex128 else C64_IR
    if lda is None:
        lda = m if amode == 0 else k
    ldb = n if ldb is None else ldb
    ldc = m if ldc is None else ldc
    _check(lib().d3m_debug_gemm(prec, m, n, k, amode, i0, _ptr(A), lda, _ptr(d) if d is not None else None,
                                _ptr(B), ldb, _ptr(C), ldc, float(alpha), float(beta), _stream(stream)),
           "d3m_debug_gemm")
    return C


def device_ok() -> bool:
    return bool(lib().d3m_device_ok())


def analyze(sizes, pairs, order=None, grid=None, **kw) -> Plan:
    return Plan(sizes, pairs, order=order, grid=grid, **kw)


class Batch:
    """Many bound factors run as one persistent launch per phase."""

    def __init__(self, factors: Sequence[Factor]):
        import torch
        self.factors = list(factors)
        n = len(self.factors)
        arr = (_vp * n)(*[f._h for f in self.factors])
        b = ctypes.c_size_t()
        _check(lib().d3m_batch_workspace_bytes(n, arr, ctypes.byref(b)), "d3m_batch_workspace_bytes")
        self.ws = torch.empty(b.value + 256, dtype=torch.uint8, device=torch.device("cuda", torch.cuda.current_device()))
        off = (-self.ws.data_ptr()) % 256
        h = _vp()
        _check(lib().d3m_batch_create(n, arr, ctypes.c_void_p(self.ws.data_ptr() + off), b.value, ctypes.byref(h)),
               "d3m_batch_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and h.value and _LIB is not None:
            _LIB.d3m_batch_destroy(h)
            self._h = None

    def run(self, Ks, Bs, Xs, stream=None):
        n = len(self.factors)
        for f, K, B in zip(self.factors, Ks, Bs):
            f._checkK(K)
            f._checkB(B)
            f.K = K
        kp = (_vp * n)(*[K.data_ptr() for K in Ks])
        bp = (_vp * n)(*[B.data_ptr() for B in Bs])
        xp = (_vp * n)(*[X.data_ptr() for X in Xs])
        nr = np.asarray([B.shape[0] for B in Bs], dtype=np.int32)
        ld = np.asarray([B.stride(0) for B in Bs], dtype=np.int64)
        _check(lib().d3m_batch_run(self._h, kp, bp, xp, _p32(nr), ld.ctypes.data_as(_i64p), _stream(stream)),
               "d3m_batch_run")
        return Xs


def gemm_candidates(precision: int = C128) -> dict:
    """Measured aggregate GFLOP/s of the task-body GEMM along each candidate
    load path (d3m_tune_gemm): {"rates": [update direct/register, update
    half-depth register, solve whole-k, solve split-k], "best": index of the
    faster update-tile candidate}."""
    import torch
    es = 16 if precision == C128 else 8
    nbytes = 256 * 3 * 128 * 512 * es
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    best = _i32()
    nc = _i32()
    g = (ctypes.c_double * 8)()
    _check(lib().d3m_tune_gemm(int(precision), _ptr(buf), nbytes, ctypes.byref(best), g, ctypes.byref(nc)),
           "d3m_tune_gemm")
    return {"rates": [float(g[i]) for i in range(nc.value)], "best": int(best.value)}


def gemm_rate(precision: int = C128) -> float:
    """Measured aggregate GFLOP/s of the factor's update-tile GEMM path
    (256 workgroups, each repeating 128x128x512 complex tile products)."""
    return gemm_candidates(precision)["rates"][0]
