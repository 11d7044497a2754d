"""Python front of the CPU FP64 oracle (ctypes over liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The GPU library never imports it.

The oracle computes X = K^{-1} B for the block-sparse complex-symmetric
reduced matrix K of D3M (Sec. II of the paper, dual factorization and
solution) through a plain block LDL^T without pivoting; see oracle.cpp.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        lib.orc_grid_interfaces.restype = ctypes.c_int32
        lib.orc_grid_interfaces.argtypes = [_i32p, _i32p]
        lib.orc_grid_pairs.restype = ctypes.c_int64
        lib.orc_grid_pairs.argtypes = [_i32p, _i32p]
        lib.orc_nd_order.restype = ctypes.c_int32
        lib.orc_nd_order.argtypes = [_i32p, _i32p]
        lib.orc_plan.restype = ctypes.c_void_p
        lib.orc_plan.argtypes = [ctypes.c_int32, _i32p, ctypes.c_int64, _i32p, _i32p]
        lib.orc_plan_free.restype = None
        lib.orc_plan_free.argtypes = [ctypes.c_void_p]
        lib.orc_plan_stats.restype = None
        lib.orc_plan_stats.argtypes = [ctypes.c_void_p, _i64p, _f64p]
        lib.orc_plan_struct.restype = ctypes.c_int32
        lib.orc_plan_struct.argtypes = [ctypes.c_void_p, ctypes.c_int32, _i32p]
        lib.orc_factor.restype = ctypes.c_int64
        lib.orc_factor.argtypes = [ctypes.c_void_p, _f64p]
        lib.orc_get_block.restype = ctypes.c_int32
        lib.orc_get_block.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, _f64p]
        lib.orc_factor_bk.restype = ctypes.c_int64
        lib.orc_factor_bk.argtypes = [ctypes.c_void_p, _f64p, ctypes.c_int32]
        lib.orc_get_pivots.restype = ctypes.c_int32
        lib.orc_get_pivots.argtypes = [ctypes.c_void_p, ctypes.c_int32, _i32p, _f64p]
        lib.orc_solve.restype = None
        lib.orc_solve.argtypes = [ctypes.c_void_p, _f64p, _f64p, ctypes.c_int32]
        lib.orc_matvec.restype = None
        lib.orc_matvec.argtypes = [ctypes.c_int32, _i32p, ctypes.c_int64, _i32p, _f64p, _f64p,
                                   _f64p, ctypes.c_int32]
        lib.orc_grad_K.restype = None
        lib.orc_grad_K.argtypes = [ctypes.c_int32, _i32p, ctypes.c_int64, _i32p, _f64p, _f64p,
                                   _f64p, ctypes.c_int32]
        _LIB = lib
    return _LIB


def _p(a, t):
    return a.ctypes.data_as(t)


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _c128(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def grid_interfaces(grid):
    g = _i32(grid)
    nb = _lib().orc_grid_interfaces(_p(g, _i32p), None)
    out = np.zeros((nb, 4), dtype=np.int32)
    _lib().orc_grid_interfaces(_p(g, _i32p), _p(out, _i32p))
    return out


def grid_pairs(grid):
    g = _i32(grid)
    npair = _lib().orc_grid_pairs(_p(g, _i32p), None)
    out = np.zeros((npair, 2), dtype=np.int32)
    _lib().orc_grid_pairs(_p(g, _i32p), _p(out, _i32p))
    return out


def nd_order(grid):
    g = _i32(grid)
    nb = _lib().orc_grid_interfaces(_p(g, _i32p), None)
    out = np.zeros(nb, dtype=np.int32)
    k = _lib().orc_nd_order(_p(g, _i32p), _p(out, _i32p))
    assert k == nb
    return out


class OraclePlan:
    """Symbolic block factorization for a given elimination order."""

    def __init__(self, sizes, pairs, order):
        self.sizes = _i32(sizes)
        self.pairs = _i32(np.asarray(pairs).reshape(-1, 2))
        self.order = _i32(order)
        self.nb = int(self.sizes.shape[0])
        self.N = int(self.sizes.astype(np.int64).sum())
        self._h = _lib().orc_plan(self.nb, _p(self.sizes, _i32p), int(self.pairs.shape[0]),
                                  _p(self.pairs, _i32p), _p(self.order, _i32p))
        self.pivot_index = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib().orc_plan_free(h)
            self._h = None

    def stats(self) -> dict:
        st = np.zeros(16, dtype=np.int64)
        fl = np.zeros(4, dtype=np.float64)
        _lib().orc_plan_stats(self._h, _p(st, _i64p), _p(fl, _f64p))
        keys = ["N", "fill_blocks", "L_blocks", "nnz_L", "fact_tasks", "trsm_tasks",
                "update_tasks", "etree_height", "max_S", "max_degree"]
        d = {k: int(st[i]) for i, k in enumerate(keys)}
        d.update(flops_diag=float(fl[0]), flops_trsm=float(fl[1]), flops_update=float(fl[2]),
                 flops=float(fl[3]))
        return d

    def struct(self, I: int) -> list:
        out = np.zeros(self.nb, dtype=np.int32)
        k = _lib().orc_plan_struct(self._h, int(I), _p(out, _i32p))
        return out[:k].tolist()

    def factor(self, K) -> int:
        """Returns -1, or the global row of the first zero/non-finite pivot."""
        K = _c128(K)
        r = int(_lib().orc_factor(self._h, _p(K.view(np.float64), _f64p)))
        self.pivot_index = None if r < 0 else r
        return r

    def factor_bk(self, K, tile: int = 128) -> int:
        """Factor with Bunch-Kaufman pivoting restricted to segments of `tile`
        unknowns of each interface.  Returns -1, or the global row of the
        first zero pivot column."""
        K = _c128(K)
        r = int(_lib().orc_factor_bk(self._h, _p(K.view(np.float64), _f64p), int(tile)))
        self.pivot_index = None if r < 0 else r
        return r

    def pivots(self, I: int):
        """(perm, doff) of interface I after factor_bk: internal position ->
        original index inside I, and D's off-diagonal entries (doff[k] =
        D(k+1, k) when a 2x2 pivot starts at k, else 0)."""
        n = int(self.sizes[I])
        perm = np.zeros(n, dtype=np.int32)
        doff = np.zeros(n, dtype=np.complex128)
        if _lib().orc_get_pivots(self._h, int(I), _p(perm, _i32p), _p(doff.view(np.float64), _f64p)) != 0:
            raise ValueError("no pivots: factor with factor_bk")
        return perm, doff

    def block(self, J: int, I: int) -> np.ndarray:
        nJ, nI = int(self.sizes[J]), int(self.sizes[I])
        out = np.zeros(nJ * nI, dtype=np.complex128)
        r = _lib().orc_get_block(self._h, int(J), int(I), _p(out.view(np.float64), _f64p))
        if r != 0:
            raise KeyError((J, I))
        return out.reshape(nJ, nI, order="F")

    def solve(self, B) -> np.ndarray:
        B = _c128(B)
        if B.ndim == 1:
            B = B.reshape(1, -1)
        m = B.shape[0]
        assert B.shape[1] == self.N
        X = np.zeros_like(B)
        _lib().orc_solve(self._h, _p(B.view(np.float64), _f64p), _p(X.view(np.float64), _f64p), m)
        return X


def matvec(sizes, pairs, K, X) -> np.ndarray:
    sizes, pairs = _i32(sizes), _i32(np.asarray(pairs).reshape(-1, 2))
    K, X = _c128(K), _c128(X)
    if X.ndim == 1:
        X = X.reshape(1, -1)
    Y = np.zeros_like(X)
    _lib().orc_matvec(int(sizes.shape[0]), _p(sizes, _i32p), int(pairs.shape[0]), _p(pairs, _i32p),
                      _p(K.view(np.float64), _f64p), _p(X.view(np.float64), _f64p),
                      _p(Y.view(np.float64), _f64p), X.shape[0])
    return Y


def grad_K(sizes, pairs, Lam, X, klen: int) -> np.ndarray:
    sizes, pairs = _i32(sizes), _i32(np.asarray(pairs).reshape(-1, 2))
    Lam, X = _c128(Lam), _c128(X)
    if X.ndim == 1:
        X, Lam = X.reshape(1, -1), Lam.reshape(1, -1)
    dK = np.zeros(klen, dtype=np.complex128)
    _lib().orc_grad_K(int(sizes.shape[0]), _p(sizes, _i32p), int(pairs.shape[0]), _p(pairs, _i32p),
                      _p(Lam.view(np.float64), _f64p), _p(X.view(np.float64), _f64p),
                      _p(dK.view(np.float64), _f64p), X.shape[0])
    return dK


def backward_error(sizes, pairs, K, X, B, knorm_inf: float | None = None) -> np.ndarray:
    """Normwise backward error per column: ||b - Kx||_inf / (||K||_inf ||x||_inf + ||b||_inf)."""
    R = _c128(B) - matvec(sizes, pairs, K, X)
    if knorm_inf is None:
        knorm_inf = k_norm_inf(sizes, pairs, K)
    num = np.abs(R).max(axis=1)
    den = knorm_inf * np.abs(X).max(axis=1) + np.abs(B).max(axis=1)
    return num / den


def k_norm_inf(sizes, pairs, K) -> float:
    """Max row sum of |k_ij| over the full symmetric K."""
    sizes = np.asarray(sizes, dtype=np.int64)
    pairs = np.asarray(pairs).reshape(-1, 2)
    nb = sizes.shape[0]
    row0 = np.zeros(nb + 1, dtype=np.int64)
    row0[1:] = np.cumsum(sizes)
    rs = np.zeros(int(row0[-1]))
    o = 0
    for i in range(nb):
        n = int(sizes[i])
        A = np.abs(np.asarray(K[o:o + n * n]).reshape(n, n, order="F"))
        A = np.tril(A) + np.tril(A, -1).T
        rs[row0[i]:row0[i + 1]] += A.sum(axis=1)
        o += n * n
    for i, j in pairs.tolist():
        ni, nj = int(sizes[i]), int(sizes[j])
        A = np.abs(np.asarray(K[o:o + ni * nj]).reshape(ni, nj, order="F"))
        rs[row0[i]:row0[i + 1]] += A.sum(axis=1)
        rs[row0[j]:row0[j + 1]] += A.sum(axis=0)
        o += ni * nj
    return float(rs.max())
