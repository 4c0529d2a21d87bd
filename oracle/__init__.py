"""CPU oracle for the sparse LU hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product library never loads it.

``gp_oracle.c`` holds the plain FP64 Gilbert-Peierls LU with threshold
pivoting, the two triangular solves, the level computation, a brute-force
column elimination tree and the restart closure; ``dense.py`` holds a dense
NumPy checker of the same pivoting rule used to pin the sparse oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, STRUCT_SINGULAR, NUM_SINGULAR, NOMEM, BADARG = 0, -1, -2, -3, -4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU involved)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _OrLu(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("status", ctypes.c_int), ("fail_col", ctypes.c_int),
                ("nswaps", ctypes.c_int),
                ("pivrow", ctypes.POINTER(ctypes.c_int)),
                ("Lp", ctypes.POINTER(ctypes.c_int)), ("Li", ctypes.POINTER(ctypes.c_int)),
                ("Lx", ctypes.POINTER(ctypes.c_double)),
                ("Up", ctypes.POINTER(ctypes.c_int)), ("Ui", ctypes.POINTER(ctypes.c_int)),
                ("Ux", ctypes.POINTER(ctypes.c_double))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        lib.or_gp_lu.argtypes = [ctypes.c_int, ip, ip, dp, ip, ip, ctypes.c_double,
                                 ctypes.c_void_p, ctypes.POINTER(_OrLu)]
        lib.or_gp_lu.restype = ctypes.c_int
        lib.or_lu_free.argtypes = [ctypes.POINTER(_OrLu)]
        lib.or_lsolve.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp]
        lib.or_usolve.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp]
        lib.or_utsolve.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp]
        lib.or_ltsolve.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp]
        lib.or_levels.argtypes = [ctypes.c_int, ip, ip, ip]
        lib.or_coletree.argtypes = [ctypes.c_int, ip, ip, ip]
        lib.or_coletree.restype = ctypes.c_int
        lib.or_restart_set.argtypes = [ctypes.c_int, ip, ip, ip]
        lib.or_lu_errbound.argtypes = [ctypes.c_int, ip, ip, dp, ip, ip, dp, ctypes.c_double, dp, dp]
        lib.or_lu_errbound.restype = ctypes.c_int
        lib.or_mac_count.argtypes = [ctypes.c_int, ip, ip, ip]
        lib.or_mac_count.restype = ctypes.c_double
        _lib = lib
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class LU:
    """Result of the oracle factorization.  A-hat(pivrow, :) = L U."""
    n: int
    status: int
    fail_col: int
    nswaps: int
    pivrow: np.ndarray | None
    Lp: np.ndarray | None
    Li: np.ndarray | None
    Lx: np.ndarray | None
    Up: np.ndarray | None
    Ui: np.ndarray | None
    Ux: np.ndarray | None

    @property
    def nnz_lu(self) -> int:
        """nnz(L + U - I): stored strictly-lower L plus all of U."""
        return int(self.Lp[-1] + self.Up[-1])


def gp_lu(n, colptr, rowind, values, rowperm=None, colperm=None, eps=1e-3,
          init_pivrow=None) -> LU:
    """FP64 Gilbert-Peierls LU with threshold pivoting on A(rowperm, colperm)."""
    lib = _load()
    ident = np.arange(n, dtype=np.int32)
    rp = ident if rowperm is None else _i32(rowperm)
    cp = ident if colperm is None else _i32(colperm)
    ip = None if init_pivrow is None else _i32(init_pivrow)
    res = _OrLu()
    lib.or_gp_lu(int(n), _i32(colptr), _i32(rowind), _f64(values), rp, cp, float(eps),
                 None if ip is None else ip.ctypes.data_as(ctypes.c_void_p), ctypes.byref(res))
    try:
        if res.status != OK:
            return LU(n, res.status, res.fail_col, res.nswaps, None, None, None, None, None, None, None)
        lp = np.ctypeslib.as_array(res.Lp, (n + 1,)).copy()
        up = np.ctypeslib.as_array(res.Up, (n + 1,)).copy()
        nl, nu = int(lp[-1]), int(up[-1])
        li = np.ctypeslib.as_array(res.Li, (max(nl, 1),))[:nl].copy()
        lx = np.ctypeslib.as_array(res.Lx, (max(nl, 1),))[:nl].copy()
        ui = np.ctypeslib.as_array(res.Ui, (max(nu, 1),))[:nu].copy()
        ux = np.ctypeslib.as_array(res.Ux, (max(nu, 1),))[:nu].copy()
        piv = np.ctypeslib.as_array(res.pivrow, (max(n, 1),))[:n].copy()
        return LU(n, OK, -1, res.nswaps, piv, lp, li, lx, up, ui, ux)
    finally:
        lib.or_lu_free(ctypes.byref(res))


def lsolve(lu: LU, b):
    y = _f64(b).copy()
    _load().or_lsolve(lu.n, lu.Lp, lu.Li, lu.Lx, y, y)
    return y


def usolve(lu: LU, y):
    x = _f64(y).copy()
    _load().or_usolve(lu.n, lu.Up, lu.Ui, lu.Ux, x, x)
    return x


def utsolve(lu: LU, c):
    """z = U^{-T} c."""
    z = _f64(c).copy()
    _load().or_utsolve(lu.n, lu.Up, lu.Ui, lu.Ux, z, z)
    return z


def ltsolve(lu: LU, z):
    """w = L^{-T} z (unit diagonal)."""
    w = _f64(z).copy()
    _load().or_ltsolve(lu.n, lu.Lp, lu.Li, lu.Lx, w, w)
    return w


def solve_transposed(lu: LU, rowperm, colperm, c):
    """Solve A' y = c given A-hat = A(rowperm, colperm) and A-hat(pivrow,:) = L U.

    With B = A(rowperm[pivrow], colperm) = L U, B' = A'(colperm, rowperm[pivrow]),
    so y(rowperm[pivrow]) = L^{-T} U^{-T} c(colperm)."""
    rowperm = np.asarray(rowperm); colperm = np.asarray(colperm)
    w = ltsolve(lu, utsolve(lu, _f64(c)[colperm]))
    y = np.empty_like(w)
    y[rowperm[lu.pivrow]] = w
    return y


def solve(lu: LU, rowperm, colperm, b):
    """Solve A x = b given A-hat = A(rowperm, colperm) and A-hat(pivrow,:) = L U."""
    rowperm = np.asarray(rowperm); colperm = np.asarray(colperm)
    b = _f64(b)
    z = usolve(lu, lsolve(lu, b[rowperm[lu.pivrow]]))
    x = np.empty_like(z)
    x[colperm] = z
    return x


def levels(lu: LU) -> np.ndarray:
    lev = np.zeros(lu.n, dtype=np.int32)
    _load().or_levels(lu.n, lu.Up, lu.Ui, lev)
    return lev


def coletree(n, colptr, rowind) -> np.ndarray:
    """Column elimination tree of the given CSC pattern (parent array, -1 = root)."""
    par = np.full(n, -1, dtype=np.int32)
    rc = _load().or_coletree(int(n), _i32(colptr), _i32(rowind), par)
    if rc != OK:
        raise MemoryError("oracle coletree")
    return par


def restart_set(parent, unfinished) -> np.ndarray:
    parent = _i32(parent)
    out = np.zeros(parent.size, dtype=np.int32)
    _load().or_restart_set(parent.size, parent, _i32(np.asarray(unfinished, dtype=bool)), out)
    return out.astype(bool)


def lu_error_bound(lu: LU, roundings_per_product=1.0):
    """First-order rounding-error bound of every factor entry (eL, eU in the factors'
    order), from or_lu_errbound."""
    eL = np.zeros(max(int(lu.Lp[-1]), 1))
    eU = np.zeros(max(int(lu.Up[-1]), 1))
    rc = _load().or_lu_errbound(lu.n, lu.Lp, lu.Li, _f64(lu.Lx), lu.Up, lu.Ui, _f64(lu.Ux),
                                float(roundings_per_product), eL, eU)
    if rc != OK:
        raise MemoryError("oracle error bound")
    return eL[:int(lu.Lp[-1])], eU[:int(lu.Up[-1])]


def mac_count(lu: LU) -> float:
    return float(_load().or_mac_count(lu.n, lu.Lp, lu.Up, lu.Ui))


def permuted_pattern(n, colptr, rowind, rowperm, colperm):
    """CSC pattern of A-hat = A(rowperm, colperm), rows sorted."""
    rowinv = np.empty(n, dtype=np.int64)
    rowinv[np.asarray(rowperm)] = np.arange(n)
    cols, rows = [], []
    colptr = np.asarray(colptr); rowind = np.asarray(rowind)
    hp = np.zeros(n + 1, dtype=np.int32)
    for j in range(n):
        c = colperm[j]
        r = np.sort(rowinv[rowind[colptr[c]:colptr[c + 1]]])
        rows.append(r)
        hp[j + 1] = hp[j] + r.size
    hi = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    return hp, hi


def backward_error(colptr, rowind, values, x, b):
    """eta_inf = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf), FP64 (x, b may be [n] or [n, k])."""
    import scipy.sparse as sp
    n = len(colptr) - 1
    A = sp.csc_matrix((values, rowind, colptr), shape=(n, n))
    r = b - A @ x
    anorm = abs(A).sum(axis=1).max()
    return float(np.abs(r).max() / (anorm * np.abs(x).max() + np.abs(b).max()))
