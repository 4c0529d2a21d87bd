"""Dense threshold-GEPP checker -- TEST INFRASTRUCTURE ONLY.

A plain NumPy elimination on a dense copy of the pre-processed matrix, with
the same threshold rule as the sparse oracle (Section II-A, Algorithm 1):
keep the row in position k when its value is finite, nonzero and at least
eps times the largest other candidate; otherwise exchange it with the
arg-max (ties to the smallest position).  Used only on tiny matrices to pin
the sparse oracle's pivots and values by brute force.
"""
from __future__ import annotations

import numpy as np


def dense_threshold_lu(M, eps):
    """Return (pivrow, L, U) with M[pivrow] = L @ U, or raise on singularity.

    Column-by-column right-looking elimination of a dense copy; rows are
    exchanged physically, so position k always holds row pivrow[k].
    """
    M = np.array(M, dtype=np.float64)
    n = M.shape[0]
    W = M.copy()
    piv = np.arange(n)
    for k in range(n):
        col = W[k:, k]
        if not np.all(np.isfinite(col)):
            raise ZeroDivisionError("non-finite candidate at column %d" % k)
        a = np.abs(col)
        other = a[1:].max() if n - k > 1 else 0.0
        if not (col[0] != 0.0 and a[0] >= eps * other):
            p = int(np.argmax(a))          # first maximum = smallest position
            if col[p] == 0.0:
                raise ZeroDivisionError("zero pivot at column %d" % k)
            if p != 0:
                W[[k, k + p]] = W[[k + p, k]]
                piv[[k, k + p]] = piv[[k + p, k]]
        W[k + 1:, k] /= W[k, k]
        W[k + 1:, k + 1:] -= np.outer(W[k + 1:, k], W[k, k + 1:])
    L = np.tril(W, -1) + np.eye(n)
    U = np.triu(W)
    return piv, L, U


def symbolic_pattern(Mbool, pivrow):
    """Boolean elimination with a fixed pivot sequence: the fill pattern of L+U.

    Entries are structurally nonzero after step k when they were nonzero or
    when both L(i,k) and U(k,j) are structurally nonzero.
    """
    S = np.array(Mbool, dtype=bool)[np.asarray(pivrow)].copy()
    n = S.shape[0]
    for k in range(n):
        rows = np.nonzero(S[k + 1:, k])[0] + k + 1
        cols = np.nonzero(S[k, k + 1:])[0] + k + 1
        if rows.size and cols.size:
            S[np.ix_(rows, cols)] = True
    return S
