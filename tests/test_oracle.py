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


# ---------------------------------------------------------------- MAC count
def _dense_macs(n):
    """Multiply-adds of a dense n x n LU: sum over pivot j of (n-1-j)^2."""
    return (n - 1) * n * (2 * n - 1) // 6


def test_oracle_mac_count_closed_forms(oracle_mod):
    """or_mac_count against closed forms: dense (and arrow with its hub first, which
    fills completely) sum_{m<n} m^2; tridiagonal and arrow-last n-1; diagonal 0."""
    for n in (1, 2, 3, 7, 12, 20):
        for kind, want in (("dense", _dense_macs(n)), ("arrow_first", _dense_macs(n)),
                           ("tridiagonal", n - 1), ("arrow_last", n - 1), ("diagonal", 0)):
            c = mnagen.hand_pattern(kind, n)
            lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values)
            assert lu.status == 0
            assert oracle_mod.mac_count(lu) == want, (kind, n)


def _triple_count(Lb, Ub):
    """#{(i, j, k): L(i,j) != 0, i > j, U(j,k) != 0, k > j} by explicit loops."""
    n = Lb.shape[0]
    cnt = 0
    for j in range(n):
        for i in range(j + 1, n):
            if not Lb[i, j]:
                continue
            for k in range(j + 1, n):
                if Ub[j, k]:
                    cnt += 1
    return cnt


@pytest.mark.parametrize("eps", [1.0, 0.1, 1e-3])
def test_oracle_mac_count_bruteforce(oracle_mod, eps):
    """or_mac_count equals a brute-force triple count over the fill pattern that a
    dense boolean elimination with the dense checker's pivots produces: every
    (i, j, k) with L(i,j) and U(j,k) structurally nonzero is one multiply-add of
    the update of column k by column j."""
    for seed in range(30):
        n = 3 + seed % 14
        c = mnagen.random_pattern(n, 0.3, 4000 + seed)
        A = c.to_scipy().toarray()
        piv, _, _ = dense_threshold_lu(A, eps)
        S = symbolic_pattern(A != 0, piv)
        Lb, Ub = np.tril(S, -1), np.triu(S, 1)
        lu = oracle_mod.gp_lu(n, c.colptr, c.rowind, c.values, eps=eps)
        assert lu.status == 0
        assert oracle_mod.mac_count(lu) == _triple_count(Lb, Ub), seed


# ------------------------------------------------- initial pivot sequence
@pytest.mark.parametrize("eps", [1.0, 0.1, 1e-3])
def test_oracle_init_pivrow_vs_dense_bruteforce(oracle_mod, eps):
    """Re-factorization from a given pivot sequence p0 (Section II-A: the preferred
    row of column k is the row in position k): the oracle must equal the dense
    checker run on A(p0, :) from the identity, composed with p0 -- pivots exactly,
    values to rounding, pattern by boolean elimination.  Random p0 put rows with
    small or structurally zero entries in preferred positions, so exchanges happen."""
    rng = np.random.default_rng(17)
    swaps = cases_with_swaps = 0
    for seed in range(60):
        n = 3 + seed % 14
        c = mnagen.random_pattern(n, 0.3, 3000 + seed)
        A = c.to_scipy().toarray()
        p0 = rng.permutation(n).astype(np.int32)
        lu = oracle_mod.gp_lu(n, c.colptr, c.rowind, c.values, eps=eps, init_pivrow=p0)
        try:
            piv, L, U = dense_threshold_lu(A[p0], eps)
        except ZeroDivisionError:
            assert lu.status != 0
            continue
        assert lu.status == 0
        assert np.array_equal(lu.pivrow, p0[piv]), (seed, lu.pivrow, p0[piv])
        Ls, Us = _lu_dense(lu)
        assert np.abs(Ls - L).max() <= 1e-13 * max(1.0, np.abs(L).max())
        assert np.abs(Us - U).max() <= 1e-13 * max(1.0, np.abs(L).max() * np.abs(U).max())
        assert np.array_equal(_pattern(lu), symbolic_pattern(A[p0] != 0, piv))
        swaps += lu.nswaps
        cases_with_swaps += lu.nswaps > 0
    assert cases_with_swaps >= 30, cases_with_swaps


def test_oracle_refactor_exchange_vs_dense(oracle_mod):
    """A re-factorization whose check fails: factor, shrink the pivot of one column
    so its previous pivot row fails the threshold test, re-factor from the previous
    sequence; the exchange and every later column must equal the dense checker's
    elimination of A_new(previous sequence, :)."""
    eps = 0.1
    done = 0
    for seed in range(40):
        n = 6 + seed % 10
        c = mnagen.random_pattern(n, 0.35, 5000 + seed)
        A = c.to_scipy().toarray()
        lu0 = oracle_mod.gp_lu(n, c.colptr, c.rowind, c.values, eps=eps)
        if lu0.status != 0:
            continue
        # scale the entry that holds the pivot of a middle column down by 1e6
        k = n // 2
        r = lu0.pivrow[k]
        v = c.values.copy()
        lo, hi = c.colptr[k], c.colptr[k + 1]
        hit = np.nonzero(c.rowind[lo:hi] == r)[0]
        if hit.size == 0:
            continue
        v[lo + hit[0]] *= 1e-6
        A1 = A.copy()
        A1[r, k] *= 1e-6
        lu1 = oracle_mod.gp_lu(n, c.colptr, c.rowind, v, eps=eps, init_pivrow=lu0.pivrow)
        try:
            piv, L, U = dense_threshold_lu(A1[lu0.pivrow], eps)
        except ZeroDivisionError:
            assert lu1.status != 0
            continue
        assert lu1.status == 0
        assert np.array_equal(lu1.pivrow, lu0.pivrow[piv])
        Ls, Us = _lu_dense(lu1)
        assert np.abs(Ls - L).max() <= 1e-12 * max(1.0, np.abs(L).max())
        assert np.abs(Us - U).max() <= 1e-12 * max(1.0, np.abs(L).max() * np.abs(U).max())
        done += lu1.nswaps > 0
    assert done >= 10, done


# ------------------------------------------------------ transposed solves
def test_oracle_transposed_solves_exact_integer(oracle_mod):
    """U' z = c and L' w = z on exact integer unit/±1-diagonal factors (exact in FP64)."""
    rng = np.random.default_rng(5)
    n = 30
    L = np.tril(rng.integers(-2, 3, (n, n)) * (rng.uniform(size=(n, n)) < 0.2), -1) + np.eye(n)
    U = np.triu(rng.integers(-2, 3, (n, n)) * (rng.uniform(size=(n, n)) < 0.2), 1) + \
        np.diag(rng.choice([-1.0, 1.0], n))
    w = rng.integers(-3, 4, n).astype(float)
    z = L.T @ w
    cvec = U.T @ z
    assert np.abs(cvec).max() < 2 ** 40
    Ls = sp.csc_matrix(np.tril(L, -1)); Us = sp.csc_matrix(U)
    lu = oracle_mod.LU(n, 0, -1, 0, np.arange(n, dtype=np.int32),
                       Ls.indptr.astype(np.int32), Ls.indices.astype(np.int32), Ls.data,
                       Us.indptr.astype(np.int32), Us.indices.astype(np.int32), Us.data)
    assert np.array_equal(oracle_mod.utsolve(lu, cvec), z)
    assert np.array_equal(oracle_mod.ltsolve(lu, z), w)


def test_oracle_solve_transposed_vs_numpy(oracle_mod):
    c = mnagen.mesh_vsrc(8, 8, 4, seed=3)
    rng = np.random.default_rng(1)
    rp = rng.permutation(c.n); cp = rng.permutation(c.n)
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, rp, cp, eps=1e-3)
    assert lu.status == 0
    y = oracle_mod.solve_transposed(lu, rp, cp, c.rhs[0])
    yr = np.linalg.solve(c.to_scipy().toarray().T, c.rhs[0])
    assert np.abs(y - yr).max() <= 1e-8 * np.abs(yr).max()


def test_condest_vs_exact_inverse_norm(oracle_mod):
    """Hager's estimate of ||A^{-1}||_inf from the oracle's solves is a lower bound of
    the exact value (dense inverse), within a factor 3 of it on these matrices, and
    exact on at least half of them."""
    from oracle.condest import kappa_inf
    exact_hits = 0
    cases = 0
    for seed in range(24):
        c = (mnagen.random_pattern(20 + seed, 0.15, 6000 + seed) if seed % 2 else
             mnagen.mesh_vsrc(5 + seed % 4, 5 + seed % 4, 4, seed=seed))
        lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, eps=1e-3)
        if lu.status != 0:
            continue
        idn = np.arange(c.n)
        k_est = kappa_inf(oracle_mod, lu, c.colptr, c.rowind, c.values, idn, idn)
        A = c.to_scipy().toarray()
        k_ex = np.linalg.norm(A, np.inf) * np.linalg.norm(np.linalg.inv(A), np.inf)
        assert k_est <= k_ex * (1 + 1e-8), (seed, k_est, k_ex)
        assert k_est >= k_ex / 3, (seed, k_est, k_ex)
        exact_hits += k_est >= k_ex * (1 - 1e-8)
        cases += 1
    assert cases >= 20 and exact_hits >= cases * 0.5, (exact_hits, cases)


# ------------------------------------------------------- rounding-error bound
def _extended_lu(A, piv):
    """Doolittle LU of A[piv] in extended precision (numpy longdouble, 64-bit mantissa
    on x86-64), no pivoting: the reference 'exact' factors for the bound's pin."""
    M = np.array(A, dtype=np.longdouble)[np.asarray(piv)]
    n = M.shape[0]
    for k in range(n):
        M[k + 1:, k] /= M[k, k]
        M[k + 1:, k + 1:] -= np.outer(M[k + 1:, k], M[k, k + 1:])
    return M


def _graded(n, seed):
    """A matrix whose threshold pivoting at eps = 1e-3 keeps multipliers up to ~1e3:
    a random pattern with a weak diagonal, so errors propagate through large |L|."""
    c = mnagen.random_pattern(n, 0.35, seed)
    v = c.values.copy()
    for j in range(n):
        for p in range(c.colptr[j], c.colptr[j + 1]):
            if c.rowind[p] == j:
                v[p] *= 2e-3
    c.values = v
    return c


@pytest.mark.parametrize("eps", [1.0, 0.1, 1e-3])
def test_oracle_error_bound_vs_extended_precision(oracle_mod, eps):
    """The running error bound of every factor entry holds against an extended-precision
    factorization with the same pivot sequence (|oracle - exact| <= bound), on random
    and on graded matrices whose large multipliers make inherited errors dominate; and
    it is not vacuous (relative bounds far below 1)."""
    exceeded_own = 0
    for seed in range(40):
        n = 8 + seed % 20
        c = _graded(n, 7000 + seed) if seed % 2 else mnagen.random_pattern(n, 0.3, 7000 + seed)
        lu = oracle_mod.gp_lu(n, c.colptr, c.rowind, c.values, eps=eps)
        if lu.status != 0:
            continue
        eL, eU = oracle_mod.lu_error_bound(lu, 1.0)
        X = _extended_lu(c.to_scipy().toarray(), lu.pivrow)
        lcols = np.repeat(np.arange(n), np.diff(lu.Lp))
        ucols = np.repeat(np.arange(n), np.diff(lu.Up))
        dl = np.abs(lu.Lx - X[lu.Li, lcols].astype(np.float64))
        du = np.abs(lu.Ux - X[lu.Ui, ucols].astype(np.float64))
        tiny = 1e-300
        assert np.all(dl <= eL + tiny), (seed, float((dl / np.maximum(eL, tiny)).max()))
        assert np.all(du <= eU + tiny), (seed, float((du / np.maximum(eU, tiny)).max()))
        B = (sp.csc_matrix((np.abs(lu.Lx), lu.Li, lu.Lp), shape=(n, n)) + sp.identity(n)) @ \
            sp.csc_matrix((np.abs(lu.Ux), lu.Ui, lu.Up), shape=(n, n))
        Bd = B.toarray()
        scale_u = Bd[lu.Ui, ucols]
        if seed % 2 == 0:                       # well-scaled random matrices: a tight bound
            assert float((eU / np.maximum(scale_u, tiny)).max()) < 1e-10
        # the entries' own rounding alone (2 n u times their |L||U| scale) is exceeded
        # somewhere: the inherited part of the bound is needed, not decoration
        exceeded_own += int(np.any(du > 2 * n * np.finfo(float).eps * scale_u))
    if eps < 1:
        assert exceeded_own >= 1
