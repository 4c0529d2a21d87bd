"""Pins of the CPU oracle against facts that do not come from the oracle itself.

- dense brute force with the same threshold rule (pivots exact, values to rounding);
- LAPACK getrf pivots for eps = 1 (true partial pivoting, smallest-index ties);
- boolean Gaussian elimination for the fill pattern;
- closed forms: diagonal, tridiagonal, arrow, permutation, dense, 2D Laplacian;
- exact integer triangular systems for the solves;
- brute-force longest paths for the levels (Section II-B);
- dense boolean Cholesky of A'A for the column elimination tree, and the
  George-Ng containment for arbitrary pivot sequences;
- the restart example narrated in Section IV-C.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

import mnagen
from oracle.dense import dense_threshold_lu, symbolic_pattern

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense(n, p, i, x):
    return sp.csc_matrix((x, i, p), shape=(n, n)).toarray()


def _lu_dense(lu):
    n = lu.n
    return _dense(n, lu.Lp, lu.Li, lu.Lx) + np.eye(n), _dense(n, lu.Up, lu.Ui, lu.Ux)


def _pattern(lu):
    n = lu.n
    Lb = _dense(n, lu.Lp, lu.Li, np.ones(lu.Lp[-1])) != 0
    Ub = _dense(n, lu.Up, lu.Ui, np.ones(lu.Up[-1])) != 0
    return Lb | Ub


@pytest.mark.parametrize("eps", [1.0, 0.1, 1e-3])
def test_oracle_vs_dense_bruteforce(oracle_mod, eps):
    checked = 0
    for seed in range(60):
        n = 3 + seed % 13
        c = mnagen.random_pattern(n, 0.3, seed)
        A = c.to_scipy().toarray()
        lu = oracle_mod.gp_lu(n, c.colptr, c.rowind, c.values, eps=eps)
        piv, L, U = dense_threshold_lu(A, eps)
        assert lu.status == 0
        assert np.array_equal(lu.pivrow, piv), (seed, lu.pivrow, piv)
        Ls, Us = _lu_dense(lu)
        scale = np.abs(L).max() * np.abs(U).max()
        assert np.abs(Ls - L).max() <= 1e-13 * max(1.0, np.abs(L).max())
        assert np.abs(Us - U).max() <= 1e-13 * max(1.0, scale)
        # fill pattern = boolean elimination with the same pivot sequence
        assert np.array_equal(_pattern(lu), symbolic_pattern(A != 0, piv))
        checked += 1
    assert checked == 60


def test_oracle_eps1_matches_lapack_getrf(oracle_mod):
    for seed in range(40):
        n = 4 + seed % 20
        c = mnagen.random_pattern(n, 0.35, 1000 + seed)
        A = c.to_scipy().toarray()
        lu = oracle_mod.gp_lu(n, c.colptr, c.rowind, c.values, eps=1.0)
        _, ipiv = sl.lu_factor(A)
        perm = np.arange(n)
        for i, p in enumerate(ipiv):
            perm[[i, p]] = perm[[p, i]]
        assert np.array_equal(lu.pivrow, perm)


def test_oracle_tie_break_smallest_position(oracle_mod):
    # column 0 has |x| = 2 at rows 1 and 2 and a tiny diagonal: the exchange must
    # take row 1 (smallest position), as LAPACK's first-maximum rule does.
    A = np.array([[1e-9, 1.0, 0.0], [2.0, 1.0, 1.0], [-2.0, 0.0, 3.0]])
    m = sp.csc_matrix(A)
    lu = oracle_mod.gp_lu(3, m.indptr, m.indices, m.data, eps=0.5)
    assert list(lu.pivrow[:1]) == [1]
    _, ipiv = sl.lu_factor(A)
    assert ipiv[0] == 1


def test_oracle_reconstruction_with_permutations(oracle_mod):
    rng = np.random.default_rng(7)
    for seed in range(10):
        c = mnagen.random_pattern(40, 0.08, 50 + seed)
        n = c.n
        rp = rng.permutation(n).astype(np.int32)
        cp = rng.permutation(n).astype(np.int32)
        lu = oracle_mod.gp_lu(n, c.colptr, c.rowind, c.values, rp, cp, eps=0.1)
        if lu.status != 0:
            continue
        A = c.to_scipy().toarray()
        Ahat = A[rp][:, cp]
        L, U = _lu_dense(lu)
        R = Ahat[lu.pivrow] - L @ U
        bound = 40 * n * np.finfo(float).eps * (np.abs(L) @ np.abs(U)).max()
        assert np.abs(R).max() <= bound


def test_oracle_closed_forms(oracle_mod):
    # diagonal: L = I, U = diag, one level
    c = mnagen.hand_pattern("diagonal", 12)
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values)
    assert lu.Lp[-1] == 0 and lu.Up[-1] == 12
    assert np.all(oracle_mod.levels(lu) == 0)
    # diagonally dominant tridiagonal: no fill, no exchange, a chain of levels
    c = mnagen.hand_pattern("tridiagonal", 15)
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values)
    assert lu.nswaps == 0 and np.array_equal(lu.pivrow, np.arange(15))
    assert lu.Lp[-1] == 14 and lu.Up[-1] == 15 + 14
    assert np.array_equal(oracle_mod.levels(lu), np.arange(15))
    # arrow with the dense row/column last: no fill
    c = mnagen.hand_pattern("arrow_last", 10)
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values)
    assert lu.nnz_lu == c.nnz
    # arrow with it first: complete fill
    c = mnagen.hand_pattern("arrow_first", 10)
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values)
    assert lu.nnz_lu == 10 * 10
    # dense: fill is n^2
    c = mnagen.hand_pattern("dense", 9)
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values)
    assert lu.nnz_lu == 81
    # permutation matrix: pivoting is forced and recovers the permutation
    c = mnagen.hand_pattern("permutation", 11)
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values)
    A = c.to_scipy().toarray()
    for k in range(11):
        assert A[lu.pivrow[k], k] != 0
    assert lu.Lp[-1] == 0


@pytest.mark.parametrize("side", [3, 5, 8])
def test_oracle_laplacian_natural_order_fill(oracle_mod, side):
    """5-point grid in natural order: nnz(L) from the elimination front."""
    c = mnagen.hand_pattern("laplacian2d", side * side)
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values)
    assert lu.nswaps == 0
    # first grid row: node x reaches x+2 later nodes (side for the last one);
    # interior rows reach exactly `side`; the last row reaches what is left.
    first = sum(x + 2 for x in range(side - 1)) + side
    middle = (side - 2) * side * side
    last = side * (side - 1) // 2
    assert lu.Lp[-1] == first + middle + last
    assert lu.Up[-1] == lu.Lp[-1] + c.n      # structurally symmetric, no pivoting


def test_oracle_solves_exact_integer_systems(oracle_mod):
    rng = np.random.default_rng(3)
    n = 30
    L = np.tril(rng.integers(-2, 3, (n, n)) * (rng.uniform(size=(n, n)) < 0.2), -1) + np.eye(n)
    U = np.triu(rng.integers(-2, 3, (n, n)) * (rng.uniform(size=(n, n)) < 0.2), 1) + \
        np.diag(rng.choice([-1.0, 1.0], n))
    x = rng.integers(-3, 4, n).astype(float)
    y = U @ x
    b = L @ y
    assert np.abs(b).max() < 2 ** 40          # exact in FP64
    Ls = sp.csc_matrix(np.tril(L, -1)); Us = sp.csc_matrix(U)
    lu = oracle_mod.LU(n, 0, -1, 0, np.arange(n, dtype=np.int32),
                       Ls.indptr.astype(np.int32), Ls.indices.astype(np.int32), Ls.data,
                       Us.indptr.astype(np.int32), Us.indices.astype(np.int32), Us.data)
    # diagonal must be stored last in each U column
    assert all(Us.indices[Us.indptr[j + 1] - 1] == j for j in range(n))
    assert np.array_equal(oracle_mod.lsolve(lu, b), y)
    assert np.array_equal(oracle_mod.usolve(lu, y), x)


def test_oracle_solve_vs_numpy(oracle_mod):
    c = mnagen.mesh_vsrc(8, 8, 4, seed=2)
    rng = np.random.default_rng(0)
    rp = rng.permutation(c.n); cp = rng.permutation(c.n)
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, rp, cp, eps=1e-3)
    assert lu.status == 0
    x = oracle_mod.solve(lu, rp, cp, c.rhs[0])
    xr = np.linalg.solve(c.to_scipy().toarray(), c.rhs[0])
    assert np.abs(x - xr).max() <= 1e-8 * np.abs(xr).max()
    assert oracle_mod.backward_error(c.colptr, c.rowind, c.values, x, c.rhs[0]) < 1e-14


def _longest_paths_bruteforce(n, edges):
    lev = np.zeros(n, dtype=int)
    changed = True
    while changed:                           # Bellman-Ford relaxation to a fixpoint
        changed = False
        for j, k in edges:
            if lev[j] + 1 > lev[k]:
                lev[k] = lev[j] + 1
                changed = True
    return lev


def test_oracle_levels_bruteforce(oracle_mod):
    for seed in range(8):
        c = mnagen.random_pattern(30, 0.08, 300 + seed)
        lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, eps=0.1)
        edges = [(int(lu.Ui[p]), k) for k in range(c.n)
                 for p in range(lu.Up[k], lu.Up[k + 1]) if lu.Ui[p] < k]
        assert np.array_equal(oracle_mod.levels(lu), _longest_paths_bruteforce(c.n, edges))


def _etree_dense(Hb):
    """Dense boolean Cholesky of the pattern of H'H; parent = first subdiagonal."""
    M = (Hb.T.astype(int) @ Hb.astype(int)) != 0
    n = M.shape[0]
    S = M.copy()
    parent = np.full(n, -1)
    for k in range(n):
        rows = np.nonzero(S[k + 1:, k])[0] + k + 1
        if rows.size:
            parent[k] = rows[0]
            S[np.ix_(rows, rows)] = True
    return parent


def test_oracle_coletree_vs_dense_cholesky(oracle_mod):
    for seed in range(20):
        n = 5 + seed % 25
        c = mnagen.random_pattern(n, 0.12, 500 + seed)
        par = oracle_mod.coletree(n, c.colptr, c.rowind)
        Hb = c.to_scipy().toarray() != 0
        assert np.array_equal(par, _etree_dense(Hb))


def test_oracle_coletree_bounds_any_pivot_sequence(oracle_mod):
    """George-Ng: every L(i,j), U(j,i) lies on j's path to the root, for any pivoting."""
    for seed in range(12):
        c = mnagen.random_pattern(25, 0.12, 700 + seed)
        par = oracle_mod.coletree(c.n, c.colptr, c.rowind)
        anc = [set() for _ in range(c.n)]
        for j in range(c.n):
            p = par[j]
            while p >= 0:
                anc[j].add(int(p)); p = par[p]
        for eps in (1.0, 0.5, 1e-3):
            lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, eps=eps)
            for j in range(c.n):
                for p in range(lu.Lp[j], lu.Lp[j + 1]):
                    assert int(lu.Li[p]) in anc[j]
            for k in range(c.n):
                for p in range(lu.Up[k], lu.Up[k + 1] - 1):
                    assert k in anc[int(lu.Ui[p])]


def test_oracle_restart_set_golden(oracle_mod):
    rec = {}
    with open(os.path.join(GOLDEN, "restart_example.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, vals = line.split(":")
            rec[key] = [int(v) for v in vals.split()]
    parent = np.array([p - 1 for p in rec["parent"]])       # 1-based, 0 = root
    unfinished = np.zeros(10, dtype=bool)
    unfinished[np.array(rec["unfinished"]) - 1] = True
    got = np.nonzero(oracle_mod.restart_set(parent, unfinished))[0] + 1
    assert list(got) == rec["restart"]


def test_oracle_refactor_keeps_sequence_and_detects_failure(oracle_mod):
    c = mnagen.mesh_vsrc(6, 6, 4, seed=1)
    lu0 = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, eps=1e-3)
    assert lu0.status == 0 and lu0.nswaps > 0       # zero-diagonal sources force exchanges
    lu1 = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values * 1.01, eps=1e-3,
                           init_pivrow=lu0.pivrow)
    assert lu1.nswaps == 0 and np.array_equal(lu1.pivrow, lu0.pivrow)
    assert np.array_equal(lu1.Li, lu0.Li) and np.array_equal(lu1.Ui, lu0.Ui)
    # starting again from the identity re-does the exchanges
    lu2 = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values * 1.01, eps=1e-3)
    assert lu2.nswaps == lu0.nswaps


def test_oracle_singular_cases(oracle_mod):
    # structurally singular: an empty column
    A = sp.csc_matrix(np.array([[1.0, 0.0], [1.0, 0.0]]))
    lu = oracle_mod.gp_lu(2, A.indptr, A.indices, A.data)
    assert lu.status == oracle_mod.STRUCT_SINGULAR and lu.fail_col == 1
    # numerically singular: exact zero after elimination
    A = sp.csc_matrix(np.array([[1.0, 2.0], [1.0, 2.0]]))
    lu = oracle_mod.gp_lu(2, A.indptr, A.indices, A.data)
    assert lu.status == oracle_mod.NUM_SINGULAR and lu.fail_col == 1
    # non-finite value
    A = sp.csc_matrix(np.array([[np.nan, 1.0], [1.0, 1.0]]))
    lu = oracle_mod.gp_lu(2, A.indptr, A.indices, A.data)
    assert lu.status == oracle_mod.NUM_SINGULAR and lu.fail_col == 0
