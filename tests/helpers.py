"""Comparison helpers shared by the parity tests (library vs CPU oracle)."""
import numpy as np
import scipy.sparse as sp

U64 = np.finfo(np.float64).eps / 2


def lu_bound(lu):
    """B = |L| |U| (dense-free, CSC) of the oracle factors, for rounding-level tolerances."""
    n = lu.n
    L = sp.csc_matrix((np.abs(lu.Lx), lu.Li, lu.Lp), shape=(n, n)) + sp.identity(n, format="csc")
    U = sp.csc_matrix((np.abs(lu.Ux), lu.Ui, lu.Up), shape=(n, n))
    return (L @ U).tocsc()


def compare_factors(f, lu, rtol):
    """Pattern bit-exact; values within rtol of the |L||U| scale of each entry.

    For U(i,k) the scale is (|L||U|)(i,k); for L(i,k) it is
    (|L||U|)(i,k) / |U(k,k)|: first-order rounding errors of an LU are bounded by
    a multiple of u times these quantities (backward error of Gaussian elimination).
    Returns the largest scaled error.
    """
    assert np.array_equal(f["Lp"], lu.Lp), "L column pointers differ"
    assert np.array_equal(f["Li"], lu.Li), "L pattern differs"
    assert np.array_equal(f["Up"], lu.Up), "U column pointers differ"
    assert np.array_equal(f["Ui"], lu.Ui), "U pattern differs"
    B = lu_bound(lu)
    n = lu.n
    diag = lu.Ux[lu.Up[1:] - 1]
    worst = 0.0
    ucols = np.repeat(np.arange(n), np.diff(lu.Up))
    uscale = np.asarray(B[lu.Ui, ucols]).ravel()
    du = np.abs(f["Ux"] - lu.Ux) / np.maximum(uscale, np.finfo(float).tiny)
    worst = max(worst, float(du.max(initial=0.0)))
    if lu.Lp[-1]:
        lcols = np.repeat(np.arange(n), np.diff(lu.Lp))
        lscale = np.asarray(B[lu.Li, lcols]).ravel() / np.abs(diag[lcols])
        dl = np.abs(f["Lx"] - lu.Lx) / np.maximum(lscale, np.finfo(float).tiny)
        worst = max(worst, float(dl.max(initial=0.0)))
    assert worst <= rtol, f"factor values differ: scaled error {worst:.3e} > {rtol:.1e}"
    return worst


def oracle_refactor(oracle_mod, c, values, an, eps, prev_pivrow):
    """The oracle's re-factorization: same pre-processing, previous pivot sequence."""
    return oracle_mod.gp_lu(c.n, c.colptr, c.rowind, values, an["rowperm_pre"], an["colperm"], eps,
                            init_pivrow=prev_pivrow)


def compare_factors_sampled(f, lu, rtol, nsample=4000, seed=0):
    """compare_factors for large factors: patterns compared in full (bit-exact),
    values on nsample random entries of L and of U, each scaled by its own
    (|L||U|)(i,k) = sum_j |L(i,j)| |U(j,k)|, formed from row i of L and column k
    of U only."""
    assert np.array_equal(f["Lp"], lu.Lp), "L column pointers differ"
    assert np.array_equal(f["Li"], lu.Li), "L pattern differs"
    assert np.array_equal(f["Up"], lu.Up), "U column pointers differ"
    assert np.array_equal(f["Ui"], lu.Ui), "U pattern differs"
    n = lu.n
    rng = np.random.default_rng(seed)
    # |L| with its unit diagonal, by rows; |U| by columns
    Lr = (sp.csc_matrix((np.abs(lu.Lx), lu.Li, lu.Lp), shape=(n, n)) + sp.identity(n, format="csc")).tocsr()
    Lr.sort_indices()
    diag = lu.Ux[lu.Up[1:] - 1]

    def scale(i, k):
        cj = Lr.indices[Lr.indptr[i]:Lr.indptr[i + 1]]
        cv = Lr.data[Lr.indptr[i]:Lr.indptr[i + 1]]
        rj = lu.Ui[lu.Up[k]:lu.Up[k + 1]]
        rv = np.abs(lu.Ux[lu.Up[k]:lu.Up[k + 1]])
        _, a, b = np.intersect1d(cj, rj, assume_unique=True, return_indices=True)
        return float((cv[a] * rv[b]).sum())

    worst = 0.0
    for Ap, Ai, Ax, Fx, is_l in ((lu.Up, lu.Ui, lu.Ux, f["Ux"], False), (lu.Lp, lu.Li, lu.Lx, f["Lx"], True)):
        m = int(Ap[-1])
        if m == 0:
            continue
        cols = np.repeat(np.arange(n), np.diff(Ap))
        for q in rng.choice(m, size=min(nsample, m), replace=False):
            i, k = int(Ai[q]), int(cols[q])
            sc = scale(i, k) / (abs(diag[k]) if is_l else 1.0)
            worst = max(worst, abs(Fx[q] - Ax[q]) / max(sc, np.finfo(float).tiny))
    assert worst <= rtol, f"factor values differ: scaled error {worst:.3e} > {rtol:.1e}"
    return worst


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
