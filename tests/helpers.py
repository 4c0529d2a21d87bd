"""Comparison helpers shared by the parity tests (library vs CPU oracle), and the circuits and
build step of the host schedule checks."""
import os
import shutil
import subprocess

import numpy as np
import scipy.sparse as sp

import mnagen

U64 = np.finfo(np.float64).eps / 2


def gamma(m):
    """gamma_m = m u / (1 - m u), the rounding bound of a sum of m products (u = 2^-53)."""
    return m * U64 / (1.0 - m * U64)


def factor_rtol(n):
    """Scale of the |L||U|-scaled differences reported next to the per-entry check (the
    rounding of one sum of up to n products: gamma_n); informational."""
    return gamma(n)


# roundings per product in the library's arithmetic: the sweep forms x_j(i) * (1/pivot_j)
# * U(j,k), the dense block products of products in its blocked updates
LIB_ROUNDINGS = 3.0


def entry_tolerances(oracle_mod, lu):
    """Per-entry tolerance of |library - oracle| for every factor entry: the sum of the
    two first-order rounding-error bounds of the running error analysis (the oracle's
    own arithmetic, one rounding per product, and the library's, LIB_ROUNDINGS), both
    accumulated through the factorization from the oracle's factors."""
    eL1, eU1 = oracle_mod.lu_error_bound(lu, 1.0)
    eL3, eU3 = oracle_mod.lu_error_bound(lu, LIB_ROUNDINGS)
    return eL1 + eL3, eU1 + eU3


def backward_rtol(n):
    """Bound of |B - L U| / (|L||U|) entrywise for computed factors of B (Gaussian
    elimination's backward error: at most gamma_m |L||U| for sums of m terms).  The
    library's sweep forms each product as x_j(i) * (1/pivot_j) * U(j,k), three
    roundings per product instead of one, hence gamma_3n."""
    return gamma(3 * n)


def solution_rtol(kappa, eta, eta_o):
    """Bound of ||x - x_o||_inf / ||x_o||_inf for two solutions with normwise backward
    errors eta and eta_o: each lies within 2 kappa eta / (1 - kappa eta) of the exact
    solution (perturbation bound for A and b both perturbed); kappa is a Hager lower
    estimate, within a factor 3 of kappa_inf on the pinned cases, so 2 * 3 = 6, plus
    a third for the 1 / (1 - kappa eta) factor while kappa eta <= 0.1."""
    return 8.0 * kappa * (eta + eta_o) + 4 * U64


def check_solution(x, xo, kappa, eta, eta_o, what=""):
    """Assert x within solution_rtol of the oracle's xo; returns the scaled ratio."""
    assert kappa * max(eta, eta_o) <= 0.1, (what, kappa, eta, eta_o)
    err = float(np.abs(np.asarray(x) - np.asarray(xo)).max() / max(np.abs(xo).max(), np.finfo(float).tiny))
    tol = solution_rtol(kappa, eta, eta_o)
    assert err <= tol, f"{what}: forward difference {err:.3e} > bound {tol:.3e} (kappa {kappa:.3e})"
    return err / tol


def kappa_est(oracle_mod, lu, c, values, an):
    """kappa_inf(A) by Hager's estimate on the oracle's factors of A (any size)."""
    from oracle.condest import kappa_inf as _kappa
    return _kappa(oracle_mod, lu, c.colptr, c.rowind, values, an["rowperm_pre"], an["colperm"])


def check_backward_factors(f, c, values, an, pivrow):
    """Reconstruction: B = A(rowperm_pre[pivrow], colperm) against L U with the
    library's factors f, entrywise within backward_rtol(n) |L||U|.  Returns the worst
    ratio |B - LU| / (backward_rtol |L||U|)."""
    n = c.n
    A = sp.csc_matrix((values, c.rowind, c.colptr), shape=(n, n))
    rp = np.asarray(an["rowperm_pre"])[np.asarray(pivrow)]
    B = A[rp][:, np.asarray(an["colperm"])].tocsc()
    L = sp.csc_matrix((f["Lx"], f["Li"], f["Lp"]), shape=(n, n)) + sp.identity(n, format="csc")
    U = sp.csc_matrix((f["Ux"], f["Ui"], f["Up"]), shape=(n, n))
    R = (B - L @ U).tocsc()
    S = (abs(L) @ abs(U)).tocsc()
    R = abs(R)
    ratio = R.multiply(S.power(-1)) if S.nnz else R
    rmax = float(ratio.max()) if ratio.nnz else 0.0
    worst = rmax / backward_rtol(n)
    assert worst <= 1.0, f"backward error {rmax:.3e} > gamma_3n {backward_rtol(n):.3e}"
    return worst


def lu_bound(lu):
    """B = |L| |U| (dense-free, CSC) of the oracle factors, for rounding-level tolerances."""
    n = lu.n
    L = sp.csc_matrix((np.abs(lu.Lx), lu.Li, lu.Lp), shape=(n, n)) + sp.identity(n, format="csc")
    U = sp.csc_matrix((np.abs(lu.Ux), lu.Ui, lu.Up), shape=(n, n))
    return (L @ U).tocsc()


def compare_factors(f, lu, oracle_mod=None, tol=None):
    """Pattern bit-exact; every value within its rounding-error tolerance.

    tol = (tL, tU) per-entry tolerances (entry_tolerances); with oracle_mod instead
    they are computed here.  Returns the worst ratio |difference| / tolerance."""
    assert np.array_equal(f["Lp"], lu.Lp), "L column pointers differ"
    assert np.array_equal(f["Li"], lu.Li), "L pattern differs"
    assert np.array_equal(f["Up"], lu.Up), "U column pointers differ"
    assert np.array_equal(f["Ui"], lu.Ui), "U pattern differs"
    if tol is None:
        if oracle_mod is None:
            import oracle as oracle_mod
        tol = entry_tolerances(oracle_mod, lu)
    tL, tU = tol
    tiny = np.finfo(float).tiny
    worst = 0.0
    for got, want, t, what in ((f["Ux"], lu.Ux, tU, "U"), (f["Lx"], lu.Lx, tL, "L")):
        if len(want) == 0:
            continue
        d = np.abs(np.asarray(got) - want)
        r = d / np.maximum(t, tiny)
        q = int(np.argmax(r))
        worst = max(worst, float(r[q]))
        assert r[q] <= 1.0, f"{what} value {q} differs by {d[q]:.3e} > tolerance {t[q]:.3e}"
    return worst


def oracle_refactor(oracle_mod, c, values, an, eps, prev_pivrow):
    """The oracle's re-factorization: same pre-processing, previous pivot sequence."""
    return oracle_mod.gp_lu(c.n, c.colptr, c.rowind, values, an["rowperm_pre"], an["colperm"], eps,
                            init_pivrow=prev_pivrow)


def compare_factors_sampled(f, lu, oracle_mod=None):
    """compare_factors for the full-size workloads: patterns bit-exact and every value
    within its per-entry rounding-error tolerance (the bound is one pass over the
    factors in the oracle's C code)."""
    return compare_factors(f, lu, oracle_mod)


def pivot_entry(c, a, k):
    """Index of the user nonzero that holds the current pivot of column k."""
    r = a["rowperm_pre"][a["pivrow"][k]]
    col = a["colperm"][k]
    lo, hi = c.colptr[col], c.colptr[col + 1]
    p = lo + int(np.searchsorted(c.rowind[lo:hi], r))
    assert c.rowind[p] == r
    return p


def kappa_inf(c, values):
    """Infinity-norm condition number of A (dense; for small n only)."""
    A = sp.csc_matrix((values, c.rowind, c.colptr), shape=(c.n, c.n)).toarray()
    return float(np.linalg.norm(A, np.inf) * np.linalg.norm(np.linalg.inv(A), np.inf))


# ---- host schedule checks (tests/schedule_check.cpp, tests/sched_sim.cpp): small circuits of
# each generator; the power grid is large enough to have heavy update groups and solve
# supernodes pulled by several units
SCHEDULE_CASES = {
    "power_grid_200x200": lambda: mnagen.power_grid(200, 200, n_src=200, nrhs=1, seed=3),
    "mesh_transistor_50x50": lambda: mnagen.mesh_transistor(50, 50, seed=5),
    "layered_rc_3x24x24": lambda: mnagen.layered_rc(24, 24, 3, seed=7),
    "mesh_vsrc_30x30": lambda: mnagen.mesh_vsrc(30, 30, n_vsrc=6, seed=2),
}

# (dense_tail_size, solve_split_entries, sweep_panel_rows): the defaults; a dense tail of 256
# with small solve units (several units per supernode) and split panels; no dense tail
SCHEDULE_KNOBS = [(0, 0, 0), (256, 64, 16), (-1, 256, 64)]

_TESTS = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_TESTS)


def write_csc_binary(path, c):
    """The host tools' matrix file: int32 n, int64 nnz, int32 colptr[n+1], int32 rowind[nnz],
    float64 values[nnz]."""
    with open(path, "wb") as f:
        np.array([c.n], dtype=np.int32).tofile(f)
        np.array([c.nnz], dtype=np.int64).tofile(f)
        np.asarray(c.colptr, dtype=np.int32).tofile(f)
        np.asarray(c.rowind, dtype=np.int32).tofile(f)
        np.asarray(c.values, dtype=np.float64).tofile(f)


def build_host_tool(tmp_path_factory, source, flags=(), tag=""):
    """Compiles tests/<source> with g++ against the in-tree libcktlu.so (its schedule builder
    and host factorization); skips when g++, the HIP headers or the library are missing."""
    import pytest
    import paper_2411_14082_amd as ck
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("g++ or the HIP headers are not available")
    if not os.path.exists(ck.LIB_PATH):
        pytest.skip("libcktlu.so is not built")
    out = str(tmp_path_factory.mktemp("hosttool") / (os.path.splitext(source)[0] + tag))
    libdir = os.path.dirname(ck.LIB_PATH)
    cmd = ["g++", "-std=c++17", "-O1", "-g", *flags, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(_ROOT, "include"), "-I" + os.path.join(_ROOT, "paper_2411_14082_amd", "csrc"),
           os.path.join(_TESTS, source), "-o", out, "-L" + libdir, "-l:libcktlu.so", "-Wl,-rpath," + libdir,
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and flags:
        pytest.skip("the sanitizer runtime is not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-4000:]
    return out
