"""CPU tests of the library's host logic, through the C ABI (no GPU calls).

- the shared library loads and exports every function declared in include/cktlu.h;
- analyze: valid permutations, zero-free diagonal, column elimination tree equal
  to the oracle's brute-force tree of the same pre-processed matrix;
- host factorization with pivoting vs the oracle: pattern, pivot sequence and
  levels bit-exact, values within rounding;
- argument, state and singularity errors.
"""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import mnagen
import paper_2411_14082_amd as ck
from helpers import compare_factors

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "cktlu.h")) as f:
        text = f.read()
    declared = set(re.findall(r"\b(cktlu_[a-z_]+)\s*\(", text))
    assert declared, "no declarations found"
    assert declared == set(ck.EXPORTS), declared ^ set(ck.EXPORTS)
    for name in declared:
        assert hasattr(ck.lib, name), name


def _analysed(c, **kw):
    s = ck.SparseLU(c.n, c.colptr, c.rowind, **kw)
    return s


CASES = [
    ("mesh_vsrc_32", lambda: mnagen.mesh_vsrc(32, 32, 4, seed=0)),
    ("mesh_transistor_30", lambda: mnagen.mesh_transistor(30, 30, seed=1)),
    ("layered_rc_3x20", lambda: mnagen.layered_rc(20, 20, 3, seed=2)),
    ("power_grid_40", lambda: mnagen.power_grid(40, 40, n_src=50, seed=3)),
    ("random_200", lambda: mnagen.random_pattern(200, 0.02, 4)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_analyze_permutations_and_etree(oracle_mod, name, make):
    c = make()
    s = _analysed(c)
    a = s.analysis(with_pivots=False)
    rp, cp = a["rowperm_pre"], a["colperm"]
    assert np.array_equal(np.sort(rp), np.arange(c.n)) and np.array_equal(np.sort(cp), np.arange(c.n))
    A = c.to_scipy().tocsr()
    H = A[rp][:, cp].tocsc()
    H.sort_indices()
    assert np.all(H.diagonal() != 0) or all(H[i, i] != 0 or (H[:, i].indices == i).any() for i in range(c.n))
    diag_present = np.array([(H.indices[H.indptr[j]:H.indptr[j + 1]] == j).any() for j in range(c.n)])
    assert diag_present.all(), "pre-processed matrix has a structurally zero diagonal"
    if c.n <= 1100:
        par = oracle_mod.coletree(c.n, H.indptr.astype(np.int32), H.indices.astype(np.int32))
        assert np.array_equal(par, a["parent"])


@pytest.mark.parametrize("eps", [1e-3, 0.1, 1.0])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_host_factorize_matches_oracle(oracle_mod, name, make, eps):
    c = make()
    s = _analysed(c, eps=eps)
    s.factorize_host(c.values)
    a = s.analysis()
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, a["rowperm_pre"], a["colperm"], eps)
    assert lu.status == 0
    assert np.array_equal(a["pivrow"], lu.pivrow)
    compare_factors(s.factors(), lu)
    assert np.array_equal(s.levels(), oracle_mod.levels(lu))
    st = s.stats()
    assert st["nnz_l"] == lu.Lp[-1] and st["nnz_u"] == lu.Up[-1]
    assert st["macs"] == oracle_mod.mac_count(lu)
    rp, cp = s.perm()
    assert np.array_equal(rp, a["rowperm_pre"][lu.pivrow])


def test_host_refactor_preferred_row_semantics(oracle_mod):
    """A second host factorization starts from the previous pivot sequence."""
    c = mnagen.random_pattern(60, 0.06, 9)
    s = _analysed(c, eps=0.5)
    s.factorize_host(c.values)
    a0 = s.analysis()
    v1 = mnagen.perturb(c.values, 9, 0, 1, rel=0.3)
    s.factorize_host(v1)
    a1 = s.analysis()
    lu0 = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, a0["rowperm_pre"], a0["colperm"], 0.5)
    lu1 = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, v1, a0["rowperm_pre"], a0["colperm"], 0.5)
    assert np.array_equal(a1["pivrow"], lu1.pivrow)
    assert lu0.status == 0


def test_amd_reduces_fill_on_grid():
    c = mnagen.hand_pattern("laplacian2d", 30 * 30)
    nat = _analysed(c, ordering=ck.CKTLU_ORDER_NATURAL)
    nat.factorize_host(c.values)
    amd = _analysed(c)
    amd.factorize_host(c.values)
    f_nat = nat.stats()["nnz_l"]
    f_amd = amd.stats()["nnz_l"]
    assert f_amd < 0.5 * f_nat, (f_amd, f_nat)


def test_errors_and_state():
    o = ck.cktlu_default_options()
    ctx = ck.cktlu_create(o)
    try:
        v = np.ones(2)
        assert ck.cktlu_factorize_host(ctx, v) == ck.CKTLU_E_STATE
        # unsorted rows
        assert ck.cktlu_analyze(ctx, 2, np.array([0, 2, 3], np.int32), np.array([1, 0, 1], np.int32)) == ck.CKTLU_E_ARG
        # out-of-range row
        assert ck.cktlu_analyze(ctx, 2, np.array([0, 1, 2], np.int32), np.array([0, 2], np.int32)) == ck.CKTLU_E_ARG
        # structurally singular: two columns share a single row
        assert ck.cktlu_analyze(ctx, 2, np.array([0, 1, 2], np.int32), np.array([0, 0], np.int32)) == \
            ck.CKTLU_E_STRUCT_SINGULAR
        # numerically singular
        A = sp.csc_matrix(np.array([[1.0, 2.0], [1.0, 2.0]]))
        assert ck.cktlu_analyze(ctx, 2, A.indptr.astype(np.int32), A.indices.astype(np.int32)) == 0
        assert ck.cktlu_factorize_host(ctx, A.data.copy()) == ck.CKTLU_E_NUM_SINGULAR
        assert ck.cktlu_solve(ctx, 1, None, 2, None, 2, None) in (ck.CKTLU_E_ARG, ck.CKTLU_E_STATE)
    finally:
        ck.cktlu_destroy(ctx)
    bad = ck.cktlu_default_options()
    bad.pivot_eps = 2.0
    with pytest.raises(ck.CktluError):
        ck.cktlu_create(bad)
    for s in range(-7, 3):
        assert ck.strerror(s)


def test_restart_closure_vs_oracle(oracle_mod):
    """The library's restart closure (Section IV-C), called through the C ABI on the
    library's own elimination tree, equals the oracle's BFS closure for random
    unfinished sets; the golden example of Section IV-C too; bad trees are refused."""
    c = mnagen.mesh_vsrc(10, 10, 4, seed=5)
    s = _analysed(c)
    par = s.analysis(with_pivots=False)["parent"]
    rng = np.random.default_rng(0)
    for frac in (0.0, 0.01, 0.05, 0.3, 1.0):
        unf = rng.uniform(size=c.n) < frac
        got = np.zeros(c.n, np.int32)
        assert ck.cktlu_restart_closure(c.n, par, unf.astype(np.int32), got) == 0
        assert np.array_equal(got.astype(bool), oracle_mod.restart_set(par, unf)), frac
    rec = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "restart_example.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, vals = line.split(":")
            rec[key] = [int(v) for v in vals.split()]
    gpar = np.array([p - 1 for p in rec["parent"]], np.int32)
    unf = np.zeros(10, np.int32)
    unf[np.array(rec["unfinished"]) - 1] = 1
    got = np.zeros(10, np.int32)
    assert ck.cktlu_restart_closure(10, gpar, unf, got) == 0
    assert list(np.nonzero(got)[0] + 1) == rec["restart"]
    bad = gpar.copy()
    bad[3] = 1                                     # parent below its child
    assert ck.cktlu_restart_closure(10, bad, unf, got) == ck.CKTLU_E_ARG
    assert ck.cktlu_restart_closure(10, None, unf, got) == ck.CKTLU_E_ARG
    # no fallback yet: the last-restart getter refuses
    assert ck.cktlu_get_last_restart(s.ctx, None, None) == ck.CKTLU_E_STATE


def test_footprint_estimate_positive():
    c = mnagen.mesh_vsrc(8, 8, 4, seed=0)
    s = _analysed(c)
    s.factorize_host(c.values)
    assert s.footprint_bytes(1) > 12 * (s.stats()["nnz_l"] + s.stats()["nnz_u"])


def _trailing_density(f, n, D):
    T = n - D
    cnt = 0
    for k in range(T, n):
        cnt += int((f["Ui"][f["Up"][k]:f["Up"][k + 1]] >= T).sum())
        cnt += int((f["Li"][f["Lp"][k]:f["Lp"][k + 1]] >= T).sum())
    return cnt / float(D * D)


def test_dense_tail_selection():
    """Trailing dense block: forced sizes are clamped to n, -1 disables it, and
    the automatic choice is the largest multiple of 64 in [256, 8192] whose
    block of L+U reaches the density threshold."""
    c = mnagen.mesh_transistor(60, 60, seed=4)
    for tail, want in [(-1, 0), (100, 100), (10 ** 6, c.n)]:
        s = ck.SparseLU(c.n, c.colptr, c.rowind, dense_tail=tail)
        s.factorize_host(c.values)
        assert s.stats()["dense_tail"] == want
    for dens in (0.2, 0.3, 0.5):
        s = ck.SparseLU(c.n, c.colptr, c.rowind, dense_tail=0, dense_tail_density=dens)
        s.factorize_host(c.values)
        D = s.stats()["dense_tail"]
        f = s.factors()
        if D:
            assert D % 64 == 0 and 256 <= D <= min(8192, c.n)
            assert _trailing_density(f, c.n, D) >= dens
        for Dl in range(max(D + 64, 256), min(8192, c.n) // 64 * 64 + 1, 64):
            assert _trailing_density(f, c.n, Dl) < dens, (dens, D, Dl)


def _sym_pattern(c, a):
    """Adjacency (no diagonal) of B + B' where B is the transversal-permuted matrix
    in analyze's numbering (B(i, j) = A(rowperm_pre[i], colperm[j]) up to the
    ordering, which is undone here to get back to B's own numbering)."""
    rp, cp = a["rowperm_pre"], a["colperm"]
    A = c.to_scipy().tocsc()
    H = A[rp][:, cp]                                   # the ordered matrix
    S = (abs(H) + abs(H.T)).tocsr()
    S.setdiag(0)
    S.eliminate_zeros()
    return S


def _chol_nnz_brute(S):
    """nnz (with the diagonal) of the Cholesky factor of pattern S in its own order,
    by elimination on boolean sets."""
    n = S.shape[0]
    adj = [set(S.indices[S.indptr[i]:S.indptr[i + 1]].tolist()) for i in range(n)]
    nnz = n
    for k in range(n):
        higher = [j for j in adj[k] if j > k]
        nnz += len(higher)
        for a_ in higher:
            for b_ in higher:
                if a_ != b_:
                    adj[a_].add(b_)
    return nnz


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_combined_ordering_auto(oracle_mod, name, make):
    """AMF and AUTO orderings: valid permutations; AUTO's symbolic fill counts
    equal a brute-force elimination of B + B' under each method's order, and AUTO
    keeps the method with the smaller count (ties: AMD); the host factorization
    under the chosen order matches the oracle."""
    c = make()
    amd = _analysed(c, ordering=ck.CKTLU_ORDER_AMD)
    amf = _analysed(c, ordering=ck.CKTLU_ORDER_AMF)
    auto = _analysed(c, ordering=ck.CKTLU_ORDER_AUTO)
    st = auto.stats()
    assert amd.stats()["ordering_used"] == ck.CKTLU_ORDER_AMD
    assert amf.stats()["ordering_used"] == ck.CKTLU_ORDER_AMF
    for s in (amd, amf, auto):
        a = s.analysis(with_pivots=False)
        assert np.array_equal(np.sort(a["colperm"]), np.arange(c.n))
    if c.n <= 1100:
        fa = _chol_nnz_brute(_sym_pattern(c, amd.analysis(with_pivots=False)))
        ff = _chol_nnz_brute(_sym_pattern(c, amf.analysis(with_pivots=False)))
        assert st["fill_amd"] == fa and st["fill_amf"] == ff, (st["fill_amd"], fa, st["fill_amf"], ff)
    fills = {ck.CKTLU_ORDER_AMD: st["fill_amd"], ck.CKTLU_ORDER_AMF: st["fill_amf"], ck.CKTLU_ORDER_ND: st["fill_nd"],
             ck.CKTLU_ORDER_ND_CAMD: st["fill_ndc"]}
    want = min(m for m, f in fills.items() if f == min(fills.values()))   # ties: the earlier method
    assert st["ordering_used"] == want
    same = _analysed(c, ordering=want)
    assert np.array_equal(auto.analysis(with_pivots=False)["colperm"], same.analysis(with_pivots=False)["colperm"])
    auto.factorize_host(c.values)
    a = auto.analysis()
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, a["rowperm_pre"], a["colperm"], 1e-3)
    assert lu.status == 0 and np.array_equal(a["pivrow"], lu.pivrow)
    compare_factors(auto.factors(), lu)


def test_nested_dissection_ordering(oracle_mod):
    """ND ordering on a grid larger than its leaf size (so it dissects): a valid
    permutation, its symbolic fill equals a brute-force elimination of B + B' in
    that order, it beats the banded natural order's fill, AUTO keeps the least of
    the three counts, and the host factorization under ND matches the oracle.  On
    a matrix no larger than a leaf, ND is AMD itself."""
    c = mnagen.power_grid(72, 72, seed=3)
    assert c.n > 4096
    nd = _analysed(c, ordering=ck.CKTLU_ORDER_ND)
    assert nd.stats()["ordering_used"] == ck.CKTLU_ORDER_ND
    a = nd.analysis(with_pivots=False)
    assert np.array_equal(np.sort(a["colperm"]), np.arange(c.n))
    fnd = _chol_nnz_brute(_sym_pattern(c, a))
    nat = _analysed(c, ordering=ck.CKTLU_ORDER_NATURAL)
    assert fnd < _chol_nnz_brute(_sym_pattern(c, nat.analysis(with_pivots=False)))
    st = _analysed(c, ordering=ck.CKTLU_ORDER_AUTO).stats()
    assert st["fill_nd"] == fnd
    fills = {ck.CKTLU_ORDER_AMD: st["fill_amd"], ck.CKTLU_ORDER_AMF: st["fill_amf"], ck.CKTLU_ORDER_ND: st["fill_nd"],
             ck.CKTLU_ORDER_ND_CAMD: st["fill_ndc"]}
    best = min(fills.values())
    assert st["ordering_used"] == min(m for m, f in fills.items() if f == best)
    nd.factorize_host(c.values)
    a = nd.analysis()
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, a["rowperm_pre"], a["colperm"], 1e-3)
    assert lu.status == 0 and np.array_equal(a["pivrow"], lu.pivrow)
    compare_factors(nd.factors(), lu)
    small = mnagen.power_grid(30, 30, seed=1)
    p_nd = _analysed(small, ordering=ck.CKTLU_ORDER_ND).analysis(with_pivots=False)["colperm"]
    p_amd = _analysed(small, ordering=ck.CKTLU_ORDER_AMD).analysis(with_pivots=False)["colperm"]
    assert np.array_equal(p_nd, p_amd)


def test_schur_parts_bookkeeping():
    """The dense block's Schur update is cut into parts: every dense column with
    bridge entries (U entries in rows < T) gets exactly one in-place part, every
    further part a scratch column, and columns without bridge entries get none.
    Without a device no slot map is built."""
    c = mnagen.mesh_transistor(40, 40, seed=31)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, dense_tail=600)
    s.factorize_host(c.values)
    st = s.stats()
    D = st["dense_tail"]
    assert D >= 600
    T = c.n - D
    f = s.factors()
    Up, Ui = f["Up"], f["Ui"]
    bridged = sum(1 for k in range(T, c.n) if np.any(Ui[Up[k]:Up[k + 1]] < T))
    assert bridged > 0
    assert st["schur_parts"] >= bridged
    assert st["schur_scratch_cols"] == st["schur_parts"] - bridged
    assert st["slot_map_entries"] == 0


def test_phase_work_counts_vs_oracle(oracle_mod):
    """The per-phase work the roofline uses: with no dense block the sweep finalises
    every factor entry and does every multiply-add of the oracle's count; with the
    whole matrix dense the dense block does; for a split the two add up (the Schur
    update carries the sparse columns' multiply-adds into dense targets' dense rows)."""
    c = mnagen.mesh_transistor(30, 30, seed=4)
    got = {}
    for tail in (-1, 10 ** 6, 200):
        s = ck.SparseLU(c.n, c.colptr, c.rowind, dense_tail=tail)
        s.factorize_host(c.values)
        a = s.analysis()
        got[tail] = s.stats()
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, a["rowperm_pre"], a["colperm"], 1e-3)
    nlu, macs = lu.nnz_lu, oracle_mod.mac_count(lu)
    st = got[-1]
    assert st["entries_sweep"] == nlu and st["entries_dense"] == 0
    assert st["macs_sweep"] == macs and st["macs_dense"] == 0 and st["macs"] == macs
    assert st["alg_bytes_refactor_sweep"] == 12 * nlu
    st = got[10 ** 6]
    assert st["entries_dense"] == nlu and st["entries_sweep"] == 0 and st["macs_dense"] == macs
    st = got[200]
    assert st["entries_sweep"] + st["entries_dense"] == nlu
    assert st["macs_sweep"] + st["macs_schur"] + st["macs_dense"] == macs


def test_nd_constrained_amd_ordering(oracle_mod):
    """ND followed by constrained AMD (Section III-A): a valid permutation whose parts keep
    the dissection's order (the separators of the plain ND order stay after the leaves they
    split, so the first node of the last separator is placed no earlier than in ND), its
    symbolic fill equals a brute-force elimination in that order, it does not exceed plain
    ND's fill on this grid, and the host factorization under it matches the oracle."""
    c = mnagen.power_grid(72, 72, seed=3)
    ndc = _analysed(c, ordering=ck.CKTLU_ORDER_ND_CAMD)
    assert ndc.stats()["ordering_used"] == ck.CKTLU_ORDER_ND_CAMD
    a = ndc.analysis(with_pivots=False)
    assert np.array_equal(np.sort(a["colperm"]), np.arange(c.n))
    f = _chol_nnz_brute(_sym_pattern(c, a))
    st = _analysed(c, ordering=ck.CKTLU_ORDER_AUTO).stats()
    assert st["fill_ndc"] == f
    assert f <= st["fill_nd"], (f, st["fill_nd"])
    # the top separator of the dissection is the same node set, eliminated last in both
    nd = _analysed(c, ordering=ck.CKTLU_ORDER_ND).analysis(with_pivots=False)["colperm"]
    pos_nd = np.empty(c.n, np.int64); pos_nd[nd] = np.arange(c.n)
    pos_c = np.empty(c.n, np.int64); pos_c[a["colperm"]] = np.arange(c.n)
    m = 60                                              # the top separator's nodes are among the last ones
    tail_nd = set(nd[-m:].tolist())
    assert all(pos_c[v] >= c.n - 2 * m for v in tail_nd)
    ndc.factorize_host(c.values)
    a = ndc.analysis()
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, a["rowperm_pre"], a["colperm"], 1e-3)
    assert lu.status == 0 and np.array_equal(a["pivrow"], lu.pivrow)
    compare_factors(ndc.factors(), lu)


def _matched_log_product(c, a):
    """sum_j ln |A(rowperm_pre[j], colperm[j])|: the log of the product of the diagonal
    magnitudes after the transversal."""
    A = c.to_scipy().tocsc()
    return float(sum(np.log(abs(A[a["rowperm_pre"][j], a["colperm"][j]])) for j in range(c.n)))


def _dominant_rows(c, seed, k=2, f=100.0):
    """The values of c with k random rows scaled by f: most column maxima then share
    a row, so the matching needs augmenting paths and potentials beyond a greedy start."""
    rng = np.random.default_rng(seed)
    rows = rng.choice(c.n, size=min(k, c.n), replace=False)
    v = c.values.copy()
    v[np.isin(c.rowind, rows)] *= f
    c.values = v
    return c


def test_static_pivoting_matching_bruteforce():
    """Maximum-product matching (Section III-A) against brute force over all permutations
    on small matrices, half of them with dominant rows (the greedy start fails there)."""
    import itertools
    checked = 0
    for seed in range(60):
        n = 3 + seed % 5
        c = mnagen.random_pattern(n, 0.5, 8000 + seed)
        if seed % 2:
            c = _dominant_rows(c, seed, k=1 + seed % 2)
        A = c.to_scipy().toarray()
        best = -np.inf
        for perm in itertools.permutations(range(n)):
            v = A[list(perm), range(n)]
            if np.all(v != 0):
                best = max(best, float(np.sum(np.log(np.abs(v)))))
        if not np.isfinite(best):
            continue
        s = ck.SparseLU(c.n, c.colptr, c.rowind, static_pivoting=1, values=c.values)
        got = _matched_log_product(c, s.analysis(with_pivots=False))
        assert abs(got - best) <= 1e-12 * max(1.0, abs(best)), (seed, got, best)
        checked += 1
    assert checked >= 45


def test_static_pivoting_matching_vs_assignment_and_scaling():
    """The matching's log-product equals scipy's linear_sum_assignment optimum on the
    costs -ln|a_ij| (zeros excluded); the scaling makes every matched entry 1 in
    magnitude and every entry at most 1."""
    from scipy.optimize import linear_sum_assignment
    for seed in range(16):
        c = mnagen.random_pattern(40 + 10 * seed, 0.05, 9000 + seed)
        if seed % 2:
            c = _dominant_rows(c, seed, k=3 + seed % 4)
        A = c.to_scipy().toarray()
        cost = np.where(A != 0, -np.log(np.abs(np.where(A != 0, A, 1.0))), 1e6)
        r, col = linear_sum_assignment(cost)
        if np.any(A[r, col] == 0):
            continue
        best = -float(cost[r, col].sum())
        s = ck.SparseLU(c.n, c.colptr, c.rowind, static_pivoting=2, values=c.values)
        a = s.analysis(with_pivots=False)
        got = _matched_log_product(c, a)
        assert abs(got - best) <= 1e-10 * max(1.0, abs(best)), (seed, got, best)
        rs, cs = s.scaling()
        As = np.abs(rs[:, None] * A * cs[None, :])
        assert As.max() <= 1 + 1e-12
        diag = As[a["rowperm_pre"], a["colperm"]]
        assert np.abs(diag - 1).max() <= 1e-12


def test_static_pivoting_factorization_vs_oracle(oracle_mod):
    """With matching and scaling the library factors S_r P A S_c: the host factorization
    equals the oracle's on that matrix (pattern and pivots exact, values within the
    per-entry bound), and a mesh with voltage sources (zero diagonal entries) needs no
    exchange any more."""
    for c in (mnagen.mesh_vsrc(12, 12, 4, seed=3), mnagen.mesh_transistor(20, 20, seed=4)):
        s = ck.SparseLU(c.n, c.colptr, c.rowind, static_pivoting=2, values=c.values)
        s.factorize_host(c.values)
        a = s.analysis()
        rs, cs = s.scaling()
        cols = np.repeat(np.arange(c.n), np.diff(c.colptr))
        vs = c.values * rs[c.rowind] * cs[cols]
        lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, vs, a["rowperm_pre"], a["colperm"], 1e-3)
        assert lu.status == 0 and np.array_equal(a["pivrow"], lu.pivrow)
        compare_factors(s.factors(), lu)
    c = mnagen.mesh_vsrc(12, 12, 4, seed=3)
    plain = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, None, None, 1e-3)
    assert plain.nswaps > 0                         # the zero diagonals of the sources force exchanges
    s = ck.SparseLU(c.n, c.colptr, c.rowind, static_pivoting=1, values=c.values)
    a = s.analysis(with_pivots=False)
    lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, c.values, a["rowperm_pre"], a["colperm"], 1e-3)
    assert lu.status == 0 and lu.nswaps == 0
