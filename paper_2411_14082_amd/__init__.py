"""Python binding of libcktlu (circuit sparse LU on MI355X / gfx950).

Thin ctypes marshalling over the C ABI declared in ``include/cktlu.h``: the
functions keep the C names, take integers and pointers (device pointers as
ints, e.g. ``tensor.data_ptr()``) and return the C status codes.  Every step of
the numerical path runs inside the library's HIP kernels.  ``SparseLU`` is a
convenience wrapper over the same calls for PyTorch tensors.

The library is built in-tree by ``paper_2411_14082_amd.build`` (or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcktlu.so")

CKTLU_OK = 0
CKTLU_W_REPIVOTED = 1
CKTLU_W_IR_FALLBACK = 2
CKTLU_E_ARG = -1
CKTLU_E_STATE = -2
CKTLU_E_STRUCT_SINGULAR = -3
CKTLU_E_NUM_SINGULAR = -4
CKTLU_E_NOMEM = -5
CKTLU_E_HIP = -6
CKTLU_E_LIMIT = -7
CKTLU_FP64 = 0
CKTLU_FP32_IR = 1
CKTLU_ORDER_AMD = 0
CKTLU_ORDER_NATURAL = 1
CKTLU_ORDER_AMF = 2
CKTLU_ORDER_AUTO = 3
CKTLU_ORDER_ND = 4
CKTLU_ORDER_ND_CAMD = 5

# every symbol the header declares (checked by the CPU test-suite)
EXPORTS = [
    "cktlu_default_options", "cktlu_create", "cktlu_destroy", "cktlu_strerror", "cktlu_set_stream",
    "cktlu_analyze", "cktlu_factorize", "cktlu_factorize_host", "cktlu_refactorize",
    "cktlu_refactorize_nocheck", "cktlu_solve", "cktlu_solve_noalloc", "cktlu_refactorize_batched",
    "cktlu_solve_batched",
    "cktlu_step_batched_graph", "cktlu_autotune",
    "cktlu_server_default_options", "cktlu_server_create", "cktlu_server_submit", "cktlu_server_poll",
    "cktlu_server_now", "cktlu_server_destroy",
    "cktlu_get_perm", "cktlu_get_analysis", "cktlu_get_factor_nnz", "cktlu_get_factors",
    "cktlu_get_levels", "cktlu_get_stats", "cktlu_get_timing", "cktlu_footprint_bytes",
    "cktlu_restart_closure", "cktlu_get_last_restart", "cktlu_analyze_values", "cktlu_get_scaling",
]


class cktlu_options(ctypes.Structure):
    _fields_ = [("pivot_eps", ctypes.c_double), ("precision", ctypes.c_int), ("ir_tol", ctypes.c_double),
                ("ir_max_iter", ctypes.c_int), ("ordering", ctypes.c_int), ("transversal", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("force_fail_col", ctypes.c_int),
                ("dense_tail_size", ctypes.c_int), ("dense_tail_density", ctypes.c_double),
                ("timing", ctypes.c_int), ("solve_chain_width", ctypes.c_int),
                ("dense_panel_width", ctypes.c_int), ("dense_lookahead", ctypes.c_int),
                ("dense_device_repivot", ctypes.c_int), ("sweep_slot_map", ctypes.c_int),
                ("sweep_supernodes", ctypes.c_int), ("static_pivoting", ctypes.c_int),
                ("sweep_panel_rows", ctypes.c_int), ("solve_split_entries", ctypes.c_int)]


class cktlu_refactor_info(ctypes.Structure):
    _fields_ = [("repivoted", ctypes.c_int), ("first_fail_col", ctypes.c_int),
                ("restart_size", ctypes.c_int), ("pattern_changed", ctypes.c_int)]


class cktlu_solve_info(ctypes.Structure):
    _fields_ = [("ir_iters", ctypes.c_int), ("backward_err", ctypes.c_double), ("used_fp64", ctypes.c_int)]


class cktlu_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz_a", ctypes.c_int64), ("nnz_l", ctypes.c_int64),
                ("nnz_u", ctypes.c_int64), ("flops", ctypes.c_double), ("macs", ctypes.c_double),
                ("levels", ctypes.c_int64), ("max_width", ctypes.c_int64), ("etree_height", ctypes.c_int64),
                ("dense_tail", ctypes.c_int64), ("n_factorize", ctypes.c_int64),
                ("n_refactorize", ctypes.c_int64), ("n_repivot", ctypes.c_int64),
                ("n_restart_cols", ctypes.c_int64), ("n_fp64_fallback_solves", ctypes.c_int64),
                ("bytes_refactor", ctypes.c_double), ("bytes_solve", ctypes.c_double),
                ("macs_sweep", ctypes.c_double), ("bytes_sweep", ctypes.c_double),
                ("flops_dense", ctypes.c_double), ("macs_schur", ctypes.c_double), ("sweep_launches", ctypes.c_int64),
                ("dense_launches", ctypes.c_int64), ("solve_launches", ctypes.c_int64),
                ("n_device_repivot", ctypes.c_int64), ("ordering_used", ctypes.c_int64),
                ("fill_amd", ctypes.c_int64), ("fill_amf", ctypes.c_int64), ("fill_nd", ctypes.c_int64),
                ("slot_map_entries", ctypes.c_int64), ("schur_parts", ctypes.c_int64),
                ("schur_scratch_cols", ctypes.c_int64), ("entries_sweep", ctypes.c_double),
                ("entries_dense", ctypes.c_double), ("macs_dense", ctypes.c_double),
                ("alg_bytes_refactor_sweep", ctypes.c_double), ("sweep_supernodes", ctypes.c_int64),
                ("sweep_levels", ctypes.c_int64), ("fill_ndc", ctypes.c_int64),
                ("n_fp32_check_retries", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class cktlu_tune_result(ctypes.Structure):
    _fields_ = [("n_tried", ctypes.c_int32), ("dense_tail", ctypes.c_int32 * 16),
                ("ms_per_step", ctypes.c_double * 16), ("best", ctypes.c_int32),
                ("n_knob_tried", ctypes.c_int32), ("knob", ctypes.c_int32 * 16),
                ("knob_value", ctypes.c_int32 * 16), ("knob_ms_per_step", ctypes.c_double * 16),
                ("sweep_supernodes", ctypes.c_int32), ("sweep_panel_rows", ctypes.c_int32),
                ("solve_split_entries", ctypes.c_int32), ("dense_panel_width", ctypes.c_int32)]


KNOB_NAMES = {0: "sweep_supernodes", 1: "sweep_panel_rows", 2: "solve_split_entries", 3: "dense_panel_width"}


class cktlu_server_options(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_double), ("lu", cktlu_options)]


class cktlu_request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("colptr", ctypes.c_void_p), ("rowind", ctypes.c_void_p),
                ("nsteps", ctypes.c_int32), ("values_dev", ctypes.c_void_p), ("b_dev", ctypes.c_void_p),
                ("x_dev", ctypes.c_void_p), ("arrival_s", ctypes.c_double), ("tag", ctypes.c_int64)]


class cktlu_request_done(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("status", ctypes.c_int), ("arrival_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("end_s", ctypes.c_double),
                ("repivots", ctypes.c_int32), ("fp64_fallbacks", ctypes.c_int32),
                ("backward_err", ctypes.c_double), ("footprint", ctypes.c_size_t)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class cktlu_timing(ctypes.Structure):
    _fields_ = [("init_ms", ctypes.c_double), ("sweep_ms", ctypes.c_double), ("dense_ms", ctypes.c_double),
                ("solve_sparse_ms", ctypes.c_double), ("solve_dense_ms", ctypes.c_double),
                ("refactors", ctypes.c_int64), ("solve_passes", ctypes.c_int64),
                ("sweep_launches", ctypes.c_int64), ("dense_launches", ctypes.c_int64),
                ("solve_sparse_launches", ctypes.c_int64), ("solve_dense_launches", ctypes.c_int64),
                ("schur_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcktlu.so is not built; run `python -m paper_2411_14082_amd.build` "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I32 = ctypes.c_int32
    lib.cktlu_default_options.argtypes = [ctypes.POINTER(cktlu_options)]
    lib.cktlu_default_options.restype = None
    lib.cktlu_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(cktlu_options)]
    lib.cktlu_destroy.argtypes = [P]
    lib.cktlu_destroy.restype = None
    lib.cktlu_strerror.argtypes = [ctypes.c_int]
    lib.cktlu_strerror.restype = ctypes.c_char_p
    lib.cktlu_set_stream.argtypes = [P, P]
    lib.cktlu_analyze.argtypes = [P, I32, P, P]
    lib.cktlu_analyze_values.argtypes = [P, I32, P, P, P]
    lib.cktlu_get_scaling.argtypes = [P, P, P]
    lib.cktlu_factorize.argtypes = [P, P]
    lib.cktlu_factorize_host.argtypes = [P, P]
    lib.cktlu_refactorize.argtypes = [P, P, ctypes.POINTER(cktlu_refactor_info)]
    lib.cktlu_refactorize_nocheck.argtypes = [P, P]
    lib.cktlu_solve.argtypes = [P, I32, P, I32, P, I32, ctypes.POINTER(cktlu_solve_info)]
    lib.cktlu_solve_noalloc.argtypes = [P, I32, P, I32, P, I32]
    lib.cktlu_refactorize_batched.argtypes = [P, I32, P, P]
    lib.cktlu_solve_batched.argtypes = [P, I32, I32, P, P, P, P]
    lib.cktlu_step_batched_graph.argtypes = [P, I32, P, P, I32, P, P, P, I32]
    lib.cktlu_autotune.argtypes = [P, I32, P, I32, ctypes.POINTER(cktlu_tune_result)]
    lib.cktlu_server_default_options.argtypes = [ctypes.POINTER(cktlu_server_options)]
    lib.cktlu_server_default_options.restype = None
    lib.cktlu_server_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(cktlu_server_options)]
    lib.cktlu_server_submit.argtypes = [P, ctypes.POINTER(cktlu_request)]
    lib.cktlu_server_poll.argtypes = [P, ctypes.POINTER(cktlu_request_done), I32, I32]
    lib.cktlu_server_now.argtypes = [P]
    lib.cktlu_server_now.restype = ctypes.c_double
    lib.cktlu_server_destroy.argtypes = [P]
    lib.cktlu_server_destroy.restype = None
    lib.cktlu_get_perm.argtypes = [P, P, P]
    lib.cktlu_get_analysis.argtypes = [P, P, P, P, P]
    lib.cktlu_get_factor_nnz.argtypes = [P, P, P]
    lib.cktlu_get_factors.argtypes = [P, I32, P, P, P, P, P, P]
    lib.cktlu_get_levels.argtypes = [P, P]
    lib.cktlu_restart_closure.argtypes = [I32, P, P, P]
    lib.cktlu_get_last_restart.argtypes = [P, P, P]
    lib.cktlu_get_stats.argtypes = [P, ctypes.POINTER(cktlu_stats)]
    lib.cktlu_get_timing.argtypes = [P, ctypes.POINTER(cktlu_timing), ctypes.c_int]
    lib.cktlu_footprint_bytes.argtypes = [P, I32]
    lib.cktlu_footprint_bytes.restype = ctypes.c_size_t
    for name in EXPORTS:
        fn = getattr(lib, name)
        if fn.restype is ctypes.c_int or name in ("cktlu_create",):
            fn.restype = ctypes.c_int
    return lib


lib = _load()


class CktluError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} ({status})")


def strerror(status: int) -> str:
    return lib.cktlu_strerror(int(status)).decode()


def _ptr(a):
    """Pointer of a numpy array, a torch tensor, an int, or None."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _check(rc, where):
    if rc < 0:
        raise CktluError(rc, where)
    return rc


# ---- functions with the C names --------------------------------------------------------------
def cktlu_default_options() -> cktlu_options:
    o = cktlu_options()
    lib.cktlu_default_options(ctypes.byref(o))
    return o


def cktlu_create(opt: cktlu_options | None = None):
    h = ctypes.c_void_p()
    rc = lib.cktlu_create(ctypes.byref(h), ctypes.byref(opt) if opt is not None else None)
    _check(rc, "cktlu_create")
    return h


def cktlu_destroy(ctx):
    lib.cktlu_destroy(ctx)


def cktlu_set_stream(ctx, stream):
    return lib.cktlu_set_stream(ctx, stream)


def cktlu_analyze(ctx, n, colptr, rowind):
    return lib.cktlu_analyze(ctx, int(n), _ptr(colptr), _ptr(rowind))


def cktlu_factorize(ctx, values_dev):
    return lib.cktlu_factorize(ctx, _ptr(values_dev))


def cktlu_factorize_host(ctx, values_host):
    return lib.cktlu_factorize_host(ctx, _ptr(values_host))


def cktlu_refactorize(ctx, values_dev, info: cktlu_refactor_info | None = None):
    return lib.cktlu_refactorize(ctx, _ptr(values_dev), ctypes.byref(info) if info is not None else None)


def cktlu_refactorize_nocheck(ctx, values_dev):
    return lib.cktlu_refactorize_nocheck(ctx, _ptr(values_dev))


def cktlu_solve(ctx, nrhs, b_dev, ldb, x_dev, ldx, info: cktlu_solve_info | None = None):
    return lib.cktlu_solve(ctx, int(nrhs), _ptr(b_dev), int(ldb), _ptr(x_dev), int(ldx),
                           ctypes.byref(info) if info is not None else None)


def cktlu_solve_noalloc(ctx, nrhs, b_dev, ldb, x_dev, ldx):
    return lib.cktlu_solve_noalloc(ctx, int(nrhs), _ptr(b_dev), int(ldb), _ptr(x_dev), int(ldx))


def cktlu_refactorize_batched(ctx, batch, values_dev, status_dev):
    return lib.cktlu_refactorize_batched(ctx, int(batch), _ptr(values_dev), _ptr(status_dev))


def cktlu_solve_batched(ctx, batch, nrhs, b_dev, x_dev, status_dev, eta_dev=None):
    return lib.cktlu_solve_batched(ctx, int(batch), int(nrhs), _ptr(b_dev), _ptr(x_dev), _ptr(status_dev),
                                   _ptr(eta_dev))


def cktlu_step_batched_graph(ctx, batch, values_dev, status_dev, nrhs, b_dev, x_dev, eta_dev=None, ir_steps=2):
    return lib.cktlu_step_batched_graph(ctx, int(batch), _ptr(values_dev), _ptr(status_dev), int(nrhs), _ptr(b_dev),
                                        _ptr(x_dev), _ptr(eta_dev), int(ir_steps))


def cktlu_autotune(ctx, batch, values_dev, reps, out: cktlu_tune_result):
    return lib.cktlu_autotune(ctx, int(batch), _ptr(values_dev), int(reps), ctypes.byref(out))


def cktlu_server_default_options() -> cktlu_server_options:
    o = cktlu_server_options()
    lib.cktlu_server_default_options(ctypes.byref(o))
    return o


def cktlu_server_create(opt: cktlu_server_options | None = None):
    h = ctypes.c_void_p()
    _check(lib.cktlu_server_create(ctypes.byref(h), ctypes.byref(opt) if opt is not None else None),
           "cktlu_server_create")
    return h


def cktlu_server_submit(srv, req: cktlu_request):
    return lib.cktlu_server_submit(srv, ctypes.byref(req))


def cktlu_server_poll(srv, max_done=64, wait_ms=0):
    buf = (cktlu_request_done * max(1, max_done))()
    k = _check(lib.cktlu_server_poll(srv, buf, int(max_done), int(wait_ms)), "cktlu_server_poll")
    return [buf[i].as_dict() for i in range(k)]


def cktlu_server_now(srv) -> float:
    return float(lib.cktlu_server_now(srv))


def cktlu_server_destroy(srv):
    lib.cktlu_server_destroy(srv)


class Server:
    """Request loop over the C server: submit(circuit pattern + device buffers), poll()."""

    def __init__(self, slots=4, hbm_budget_bytes=0.0, precision=CKTLU_FP64, eps=1e-3, ir_tol=1e-10):
        o = cktlu_server_default_options()
        o.slots = int(slots)
        o.hbm_budget_bytes = float(hbm_budget_bytes)
        o.lu.precision = precision
        o.lu.pivot_eps = eps
        o.lu.ir_tol = ir_tol
        self.h = cktlu_server_create(o)
        self._keep = {}

    def now(self):
        return cktlu_server_now(self.h)

    def submit(self, tag, n, colptr, rowind, nsteps, values_dev, b_dev, x_dev, arrival_s=None):
        cp = np.ascontiguousarray(colptr, dtype=np.int32)
        ri = np.ascontiguousarray(rowind, dtype=np.int32)
        r = cktlu_request(n=int(n), colptr=cp.ctypes.data, rowind=ri.ctypes.data, nsteps=int(nsteps),
                          values_dev=_ptr(values_dev), b_dev=_ptr(b_dev), x_dev=_ptr(x_dev),
                          arrival_s=self.now() if arrival_s is None else float(arrival_s), tag=int(tag))
        self._keep[int(tag)] = (values_dev, b_dev, x_dev)
        _check(cktlu_server_submit(self.h, r), "cktlu_server_submit")

    def poll(self, wait_ms=0, max_done=64):
        out = cktlu_server_poll(self.h, max_done, wait_ms)
        for d in out:
            self._keep.pop(d["tag"], None)
        return out

    def close(self):
        if self.h:
            cktlu_server_destroy(self.h)
            self.h = None
            self._keep.clear()


def cktlu_get_perm(ctx, rowperm, colperm):
    return lib.cktlu_get_perm(ctx, _ptr(rowperm), _ptr(colperm))


def cktlu_get_analysis(ctx, rowperm_pre, colperm, pivrow, parent):
    return lib.cktlu_get_analysis(ctx, _ptr(rowperm_pre), _ptr(colperm), _ptr(pivrow), _ptr(parent))


def cktlu_get_factor_nnz(ctx, nnz_l, nnz_u):
    return lib.cktlu_get_factor_nnz(ctx, _ptr(nnz_l), _ptr(nnz_u))


def cktlu_get_factors(ctx, instance, Lp, Li, Lx, Up, Ui, Ux):
    return lib.cktlu_get_factors(ctx, int(instance), _ptr(Lp), _ptr(Li), _ptr(Lx), _ptr(Up), _ptr(Ui), _ptr(Ux))


def cktlu_get_levels(ctx, level):
    return lib.cktlu_get_levels(ctx, _ptr(level))


def cktlu_analyze_values(ctx, n, colptr, rowind, values):
    return lib.cktlu_analyze_values(ctx, int(n), _ptr(colptr), _ptr(rowind), _ptr(values))


def cktlu_get_scaling(ctx, rscale, cscale):
    return lib.cktlu_get_scaling(ctx, _ptr(rscale), _ptr(cscale))


def cktlu_restart_closure(n, parent, unfinished, in_set):
    return lib.cktlu_restart_closure(int(n), _ptr(parent), _ptr(unfinished), _ptr(in_set))


def cktlu_get_last_restart(ctx, unfinished, in_set):
    return lib.cktlu_get_last_restart(ctx, _ptr(unfinished), _ptr(in_set))


def cktlu_get_timing(ctx, reset=0) -> cktlu_timing:
    t = cktlu_timing()
    _check(lib.cktlu_get_timing(ctx, ctypes.byref(t), int(reset)), "cktlu_get_timing")
    return t


def cktlu_get_stats(ctx) -> cktlu_stats:
    s = cktlu_stats()
    _check(lib.cktlu_get_stats(ctx, ctypes.byref(s)), "cktlu_get_stats")
    return s


def cktlu_footprint_bytes(ctx, batch=0) -> int:
    return int(lib.cktlu_footprint_bytes(ctx, int(batch)))


# ---- convenience wrapper ---------------------------------------------------------------------
class SparseLU:
    """One circuit: analyze once, then factorize / refactorize / solve.

    Host arrays are numpy; device arrays are torch tensors (float64, int32)
    on the current HIP device.  Methods raise CktluError on errors and return
    the non-negative status (0 or a warning code).
    """

    def __init__(self, n, colptr, rowind, eps=1e-3, precision=CKTLU_FP64, ordering=CKTLU_ORDER_AUTO,
                 ir_tol=1e-10, ir_max_iter=10, stream=None, transversal=1, dense_tail=None,
                 dense_tail_density=None, timing=False, solve_chain_width=None, dense_panel_width=None,
                 dense_lookahead=None, dense_device_repivot=None, sweep_slot_map=None, sweep_supernodes=None,
                 static_pivoting=None, values=None, sweep_panel_rows=None, solve_split_entries=None):
        opt = cktlu_default_options()
        opt.timing = 1 if timing else 0
        if dense_tail is not None:
            opt.dense_tail_size = int(dense_tail)
        if dense_tail_density is not None:
            opt.dense_tail_density = float(dense_tail_density)
        if solve_chain_width is not None:
            opt.solve_chain_width = int(solve_chain_width)
        if dense_panel_width is not None:
            opt.dense_panel_width = int(dense_panel_width)
        if dense_lookahead is not None:
            opt.dense_lookahead = int(dense_lookahead)
        if dense_device_repivot is not None:
            opt.dense_device_repivot = int(dense_device_repivot)
        if sweep_slot_map is not None:
            opt.sweep_slot_map = int(sweep_slot_map)
        if sweep_supernodes is not None:
            opt.sweep_supernodes = int(sweep_supernodes)
        if static_pivoting is not None:
            opt.static_pivoting = int(static_pivoting)
        if sweep_panel_rows is not None:
            opt.sweep_panel_rows = int(sweep_panel_rows)
        if solve_split_entries is not None:
            opt.solve_split_entries = int(solve_split_entries)
        opt.pivot_eps = eps
        opt.precision = precision
        opt.ordering = ordering
        opt.ir_tol = ir_tol
        opt.ir_max_iter = ir_max_iter
        opt.transversal = transversal
        opt.stream = stream
        self.ctx = cktlu_create(opt)
        self.n = int(n)
        self._colptr = np.ascontiguousarray(colptr, dtype=np.int32)
        self._rowind = np.ascontiguousarray(rowind, dtype=np.int32)
        self.nnz = int(self._colptr[-1])
        if values is None:
            _check(cktlu_analyze(self.ctx, self.n, self._colptr, self._rowind), "cktlu_analyze")
        else:
            self._values0 = np.ascontiguousarray(values, dtype=np.float64)
            _check(cktlu_analyze_values(self.ctx, self.n, self._colptr, self._rowind, self._values0),
                   "cktlu_analyze_values")

    def close(self):
        if self.ctx:
            cktlu_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def factorize(self, values_dev):
        return _check(cktlu_factorize(self.ctx, values_dev), "cktlu_factorize")

    def factorize_host(self, values_host):
        v = np.ascontiguousarray(values_host, dtype=np.float64)
        return _check(cktlu_factorize_host(self.ctx, v), "cktlu_factorize_host")

    def refactorize(self, values_dev, info=None):
        info = info if info is not None else cktlu_refactor_info()
        rc = _check(cktlu_refactorize(self.ctx, values_dev, info), "cktlu_refactorize")
        return rc, info

    def refactorize_nocheck(self, values_dev):
        return _check(cktlu_refactorize_nocheck(self.ctx, values_dev), "cktlu_refactorize_nocheck")

    def solve(self, b_dev, x_dev, nrhs=1, ldb=None, ldx=None):
        info = cktlu_solve_info()
        rc = _check(cktlu_solve(self.ctx, nrhs, b_dev, ldb or self.n, x_dev, ldx or self.n, info),
                    "cktlu_solve")
        return rc, info

    def refactorize_batched(self, batch, values_dev, status_dev):
        return _check(cktlu_refactorize_batched(self.ctx, batch, values_dev, status_dev),
                      "cktlu_refactorize_batched")

    def solve_batched(self, batch, nrhs, b_dev, x_dev, status_dev, eta_dev=None):
        return _check(cktlu_solve_batched(self.ctx, batch, nrhs, b_dev, x_dev, status_dev, eta_dev),
                      "cktlu_solve_batched")

    def step_batched_graph(self, batch, values_dev, status_dev, nrhs, b_dev, x_dev, eta_dev=None, ir_steps=2):
        return _check(cktlu_step_batched_graph(self.ctx, batch, values_dev, status_dev, nrhs, b_dev, x_dev, eta_dev,
                                               ir_steps), "cktlu_step_batched_graph")

    def autotune(self, batch, values_dev, reps=3) -> dict:
        r = cktlu_tune_result()
        _check(cktlu_autotune(self.ctx, batch, values_dev, reps, r), "cktlu_autotune")
        k, m = r.n_tried, r.n_knob_tried
        return dict(dense_tail=list(r.dense_tail[:k]), ms_per_step=list(r.ms_per_step[:k]), best=r.best,
                    best_dense_tail=r.dense_tail[r.best],
                    knob_trials=[(KNOB_NAMES[r.knob[i]], r.knob_value[i], r.knob_ms_per_step[i]) for i in range(m)],
                    kept=dict(sweep_supernodes=r.sweep_supernodes, sweep_panel_rows=r.sweep_panel_rows,
                              solve_split_entries=r.solve_split_entries, dense_panel_width=r.dense_panel_width))

    def analysis(self, with_pivots=True):
        n = self.n
        rp, cp, pv, par = (np.zeros(n, np.int32) for _ in range(4))
        _check(cktlu_get_analysis(self.ctx, rp, cp, pv if with_pivots else None, par), "cktlu_get_analysis")
        return dict(rowperm_pre=rp, colperm=cp, pivrow=pv if with_pivots else None, parent=par)

    def perm(self):
        rp = np.zeros(self.n, np.int32)
        cp = np.zeros(self.n, np.int32)
        _check(cktlu_get_perm(self.ctx, rp, cp), "cktlu_get_perm")
        return rp, cp

    def factors(self, instance=0):
        nl = np.zeros(1, np.int64)
        nu = np.zeros(1, np.int64)
        _check(cktlu_get_factor_nnz(self.ctx, nl, nu), "cktlu_get_factor_nnz")
        n = self.n
        Lp = np.zeros(n + 1, np.int32); Up = np.zeros(n + 1, np.int32)
        Li = np.zeros(max(int(nl[0]), 1), np.int32); Lx = np.zeros(max(int(nl[0]), 1))
        Ui = np.zeros(max(int(nu[0]), 1), np.int32); Ux = np.zeros(max(int(nu[0]), 1))
        _check(cktlu_get_factors(self.ctx, instance, Lp, Li, Lx, Up, Ui, Ux), "cktlu_get_factors")
        k = int(nl[0]); m = int(nu[0])
        return dict(Lp=Lp, Li=Li[:k], Lx=Lx[:k], Up=Up, Ui=Ui[:m], Ux=Ux[:m])

    def scaling(self):
        """(rscale, cscale): the factored matrix is rscale[i] A(i, j) cscale[j]."""
        r = np.zeros(self.n)
        c = np.zeros(self.n)
        _check(cktlu_get_scaling(self.ctx, r, c), "cktlu_get_scaling")
        return r, c

    def last_restart(self):
        """(unfinished, restart set) of the last pivot-check fallback, boolean arrays."""
        unf = np.zeros(self.n, np.int32)
        rs = np.zeros(self.n, np.int32)
        _check(cktlu_get_last_restart(self.ctx, unf, rs), "cktlu_get_last_restart")
        return unf.astype(bool), rs.astype(bool)

    def levels(self):
        lev = np.zeros(self.n, np.int32)
        _check(cktlu_get_levels(self.ctx, lev), "cktlu_get_levels")
        return lev

    def stats(self) -> dict:
        return cktlu_get_stats(self.ctx).as_dict()

    def timing(self, reset=False) -> dict:
        return cktlu_get_timing(self.ctx, 1 if reset else 0).as_dict()

    def footprint_bytes(self, batch=0) -> int:
        return cktlu_footprint_bytes(self.ctx, batch)
