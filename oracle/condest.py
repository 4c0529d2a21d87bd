"""Condition estimate for the tests' forward-error bounds -- TEST INFRASTRUCTURE ONLY.

The forward error of a computed solution is bounded by the condition number
times the backward error (a standard perturbation result for linear systems),
so the tests need kappa_inf(A) = ||A||_inf ||A^{-1}||_inf for matrices far too
large to invert.  ||A^{-1}||_inf equals ||A^{-T}||_1, which Hager's method
estimates from a few solves with A^{-T} and A^{-1} (Hager, "Condition estimates",
SIAM J. Sci. Stat. Comput. 5, 1984, with Higham's refinements in "FORTRAN codes
for estimating the one-norm of a real or complex matrix", ACM TOMS 14, 1988:
at most five iterations, stop when the sign vector repeats or the estimate stops
growing, then take the larger of it and the alternating-sign test vector's
estimate).  The estimate is a lower bound of the true norm and is usually exact
or within a factor of a few; the tests that use it multiply it by a safety
factor.  The solves are the oracle's own substitutions with the oracle's
factors.
"""
from __future__ import annotations

import numpy as np


def norm1_inverse_estimate(apply_inv, apply_inv_t, n, itmax=5):
    """Estimate ||M||_1 of M = apply_inv's operator, given x -> M x and x -> M' x."""
    if n == 0:
        return 0.0
    x = np.full(n, 1.0 / n)
    y = apply_inv(x)
    est = float(np.abs(y).sum())
    if n == 1:
        return est
    xi = np.where(y >= 0, 1.0, -1.0)
    z = apply_inv_t(xi)
    j = int(np.argmax(np.abs(z)))
    for _ in range(1, itmax):
        x = np.zeros(n)
        x[j] = 1.0
        y = apply_inv(x)
        est_new = float(np.abs(y).sum())
        xi_new = np.where(y >= 0, 1.0, -1.0)
        if np.array_equal(xi_new, xi) or est_new <= est:
            est = max(est, est_new)
            break
        est = est_new
        xi = xi_new
        z = apply_inv_t(xi)
        j_new = int(np.argmax(np.abs(z)))
        if abs(z[j_new]) <= z[j]:                 # ||z||_inf <= z' x with x = e_j: a local maximum
            break
        j = j_new
    # Higham's extra test vector: alternating signs with growing magnitude
    i = np.arange(n)
    alt = np.where(i % 2 == 0, 1.0, -1.0) * (1.0 + i / (n - 1.0))
    est_alt = 2.0 * float(np.abs(apply_inv(alt)).sum()) / (3.0 * n)
    return max(est, est_alt)


def kappa_inf(oracle_mod, lu, colptr, rowind, values, rowperm, colperm):
    """kappa_inf(A) = ||A||_inf * est ||A^{-1}||_inf from the oracle's factors of A.

    ||A^{-1}||_inf = ||A^{-T}||_1: the estimator runs on M = A^{-T} (x -> A^{-T} x)
    with M' = A^{-1}."""
    import scipy.sparse as sp
    n = lu.n
    A = sp.csc_matrix((values, rowind, colptr), shape=(n, n))
    anorm = float(abs(A).sum(axis=1).max()) if n else 0.0
    inv = lambda v: oracle_mod.solve(lu, rowperm, colperm, v)
    inv_t = lambda v: oracle_mod.solve_transposed(lu, rowperm, colperm, v)
    return anorm * norm1_inverse_estimate(inv_t, inv, n)
