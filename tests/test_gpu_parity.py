"""GPU parity: the HIP path through the C ABI vs the CPU oracle.

Refactorization with pivot check must reproduce the oracle's re-factorization
(started from the previous pivot sequence): pattern and pivot sequence
bit-exact, factor values within a rounding-level tolerance scaled by |L||U|.
Solves must reach eta_inf <= 1e-12 in FP64 (1e-10 with FP32 factors and FP64
refinement) and agree with the oracle's solution up to the conditioning.

`tail` selects the order of the trailing block factored densely: -1 none
(every column sparse), 64 one full panel, 100 a full and a ragged panel, 200
three full panels and a ragged one, 10**6 every column dense.
"""
import sys

import numpy as np
import pytest

import mnagen
from helpers import (check_backward_factors, check_solution, compare_factors, kappa_est, oracle_refactor,
                     pivot_entry as _pivot_entry)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = 1e-3
# factor values: per-entry rounding-error bounds (helpers.entry_tolerances, compare_factors'
# default); reconstruction: helpers.backward_rtol(n); solutions: helpers.solution_rtol


@pytest.fixture(scope="module")
def ck():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_14082_amd as m
    return m


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


SIZES = [
    ("mesh_vsrc_32", lambda: mnagen.mesh_vsrc(32, 32, 4, seed=0)),
    ("mesh_transistor_40", lambda: mnagen.mesh_transistor(40, 40, seed=1)),
    ("layered_rc_3x24", lambda: mnagen.layered_rc(24, 24, 3, seed=2)),
    ("power_grid_60", lambda: mnagen.power_grid(60, 60, n_src=50, seed=3)),
    ("random_300", lambda: mnagen.random_pattern(300, 0.01, 4)),
]


@pytest.mark.parametrize("tail", [-1, 64, 100, 200])
@pytest.mark.parametrize("name,make", SIZES, ids=[s[0] for s in SIZES])
def test_refactorize_and_solve_fp64(ck, oracle_mod, name, make, tail):
    c = make()
    say("case", name, "n", c.n, "tail", tail)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail)
    s.factorize(dev(c.values))
    a0 = s.analysis()
    prev = a0["pivrow"]
    for t in range(1, 5):
        # element re-stamping (NR-like) and the per-nonzero stress recipe, alternating
        vh = mnagen.restamp(c, 7, 0, t) if t % 2 else mnagen.perturb(c.values, 7, 0, t)
        rc, info = s.refactorize(dev(vh))
        a = s.analysis()
        lu = oracle_refactor(oracle_mod, c, vh, a0, EPS, prev)
        assert lu.status == 0
        if lu.nswaps == 0:
            assert rc == 0 and info.repivoted == 0
        assert np.array_equal(a["pivrow"], lu.pivrow)
        f = s.factors()
        w = compare_factors(f, lu)
        wb = check_backward_factors(f, c, vh, a0, a["pivrow"]) if t <= 2 else 0.0
        prev = a["pivrow"]
        b = c.rhs[0]
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
        s.solve(dev(b), x)
        torch.cuda.synchronize()
        xg = x.cpu().numpy()
        eta = oracle_mod.backward_error(c.colptr, c.rowind, vh, xg, b)
        assert eta <= 1e-12, eta
        assert s.stats()["dense_tail"] == (min(tail, c.n) if tail > 0 else 0)
        xo = oracle_mod.solve(lu, a0["rowperm_pre"], a0["colperm"], b)
        eta_o = oracle_mod.backward_error(c.colptr, c.rowind, vh, xo, b)
        assert eta_o <= 1e-12
        kap = kappa_est(oracle_mod, lu, c, vh, a0)
        wx = check_solution(xg, xo, kap, eta, eta_o, name)
        say("  step", t, "factor/tol %.2e backward/tol %.2e x/tol %.2e kappa %.2e" % (w, wb, wx, kap))


@pytest.mark.parametrize("tail", [-1, 200])
def test_refactorize_deterministic(ck, tail):
    c = mnagen.mesh_transistor(40, 40, seed=5)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail)
    s.factorize(dev(c.values))
    v = dev(mnagen.perturb(c.values, 5, 0, 1))
    s.refactorize(v)
    f1 = s.factors()
    s.refactorize(v)
    f2 = s.factors()
    assert np.array_equal(f1["Lx"], f2["Lx"]) and np.array_equal(f1["Ux"], f2["Ux"])


@pytest.mark.parametrize("tail", [-1, 100])
def test_refactorize_nocheck_equals_checked(ck, tail):
    c = mnagen.layered_rc(20, 20, 3, seed=6)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail)
    s.factorize(dev(c.values))
    v = dev(mnagen.perturb(c.values, 6, 0, 1))
    s.refactorize(v)
    f1 = s.factors()
    s.refactorize_nocheck(v)
    f2 = s.factors()
    assert np.array_equal(f1["Lx"], f2["Lx"]) and np.array_equal(f1["Ux"], f2["Ux"])


@pytest.mark.parametrize("where", ["sparse", "dense"])
def test_forced_failure_fallback(ck, oracle_mod, where):
    """Pivot check forced to fail at one column (a sparse one, or one inside the
    dense trailing block): the fallback re-factors the restart set on the host
    and the result equals the oracle's re-factorization (nothing re-pivots)."""
    c = mnagen.mesh_transistor(30, 30, seed=8)
    tail = 100
    col = c.n // 2 if where == "sparse" else c.n - tail + 37
    o = ck.cktlu_default_options()
    o.pivot_eps = EPS
    o.force_fail_col = col
    o.dense_tail_size = tail
    ctx = ck.cktlu_create(o)
    try:
        assert ck.cktlu_analyze(ctx, c.n, c.colptr, c.rowind) == 0
        assert ck.cktlu_factorize(ctx, dev(c.values)) == 0
        n = c.n
        rp, cp, pv, par = (np.zeros(n, np.int32) for _ in range(4))
        assert ck.cktlu_get_analysis(ctx, rp, cp, pv, par) == 0
        vh = mnagen.perturb(c.values, 8, 0, 1)
        info = ck.cktlu_refactor_info()
        rc = ck.cktlu_refactorize(ctx, dev(vh), info)
        assert rc == ck.CKTLU_W_REPIVOTED and info.repivoted == 1
        assert info.first_fail_col == col
        assert info.restart_size >= 1
        st = ck.cktlu_get_stats(ctx)
        assert st.n_repivot == 1 and st.dense_tail == tail
        lu = oracle_refactor(oracle_mod, c, vh, dict(rowperm_pre=rp, colperm=cp), EPS, pv)
        pv2 = np.zeros(n, np.int32)
        assert ck.cktlu_get_analysis(ctx, None, None, pv2, None) == 0
        assert np.array_equal(pv2, lu.pivrow)
        x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
        sinfo = ck.cktlu_solve_info()
        assert ck.cktlu_solve(ctx, 1, dev(c.rhs[0]), n, x, n, sinfo) == 0
        torch.cuda.synchronize()
        assert oracle_mod.backward_error(c.colptr, c.rowind, vh, x.cpu().numpy(), c.rhs[0]) <= 1e-12
    finally:
        ck.cktlu_destroy(ctx)


@pytest.mark.parametrize("device", [0, -1], ids=["device", "host"])
@pytest.mark.parametrize("tail,offs", [(100, (30,)), (300, (10, 150, 290))])
def test_value_driven_repivot_in_dense_block(ck, oracle_mod, tail, offs, device):
    """The pivots U(k,k) of columns inside the dense block shrunk to 1e-8 of their
    values (through the diagonal entries of A, which only column k's pivot sees):
    the dense pivot test fails at the first, the fallback re-pivots (the dense
    block on the device with the threshold rule, or the host GP), and pattern,
    pivot sequence and values equal the oracle's re-factorization."""
    c = mnagen.mesh_transistor(30, 30, seed=22)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail, dense_device_repivot=device)
    s.factorize(dev(c.values))
    a0 = s.analysis()
    vh = mnagen.perturb(c.values, 22, 0, 1)
    lu1 = oracle_refactor(oracle_mod, c, vh, a0, EPS, a0["pivrow"])
    assert lu1.status == 0
    assert np.array_equal(lu1.pivrow, a0["pivrow"])
    for o in offs:
        k = c.n - tail + o
        ukk = lu1.Ux[lu1.Up[k + 1] - 1]              # diagonal: last U entry of column k
        assert lu1.Ui[lu1.Up[k + 1] - 1] == k
        vh[_pivot_entry(c, a0, k)] -= ukk * (1 - 1e-8)
    lu = oracle_refactor(oracle_mod, c, vh, a0, EPS, a0["pivrow"])
    assert lu.status == 0 and lu.nswaps >= 1
    rc, info = s.refactorize(dev(vh))
    assert rc == ck.CKTLU_W_REPIVOTED and info.repivoted == 1
    assert info.first_fail_col == c.n - tail + offs[0]
    assert s.stats()["n_device_repivot"] == (1 if device == 0 else 0)
    a = s.analysis()
    assert np.array_equal(a["pivrow"], lu.pivrow)
    compare_factors(s.factors(), lu)
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    s.solve(dev(c.rhs[0]), x)
    torch.cuda.synchronize()
    assert oracle_mod.backward_error(c.colptr, c.rowind, vh, x.cpu().numpy(), c.rhs[0]) <= 1e-12


@pytest.mark.parametrize("nfail", [1, 3])
def test_value_driven_repivot_matches_oracle(ck, oracle_mod, nfail):
    """Pivots of level-0 columns shrunk by 1e-8: the GPU check must fail, the
    fallback re-pivots, and pattern + pivot sequence equal the oracle's
    re-factorization from the previous sequence; values within rounding."""
    c = mnagen.mesh_transistor(30, 30, seed=21)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS)
    s.factorize(dev(c.values))
    a0 = s.analysis()
    lev = s.levels()
    f0 = s.factors()
    nl = np.diff(f0["Lp"])
    cand = [k for k in range(c.n) if lev[k] == 0 and nl[k] > 0]
    chosen = [cand[len(cand) * (i + 1) // (nfail + 1)] for i in range(nfail)]
    vh = mnagen.perturb(c.values, 21, 0, 1)
    for k in chosen:
        vh[_pivot_entry(c, a0, k)] *= 1e-8
    lu = oracle_refactor(oracle_mod, c, vh, a0, EPS, a0["pivrow"])
    assert lu.status == 0 and lu.nswaps >= nfail
    rc, info = s.refactorize(dev(vh))
    assert rc == ck.CKTLU_W_REPIVOTED and info.repivoted == 1
    assert info.first_fail_col in chosen               # the smallest failing column of the first failing level
    a = s.analysis()
    assert np.array_equal(a["pivrow"], lu.pivrow)
    compare_factors(s.factors(), lu)
    # the next refactorization with the same values keeps the new sequence
    rc2, info2 = s.refactorize(dev(vh))
    assert rc2 == 0 and info2.repivoted == 0
    compare_factors(s.factors(), lu)
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    s.solve(dev(c.rhs[0]), x)
    torch.cuda.synchronize()
    assert oracle_mod.backward_error(c.colptr, c.rowind, vh, x.cpu().numpy(), c.rhs[0]) <= 1e-12


@pytest.mark.parametrize("tail", [-1, 100])
@pytest.mark.parametrize("nrhs", [1, 3, 8])
def test_multi_rhs(ck, oracle_mod, nrhs, tail):
    c = mnagen.power_grid(50, 50, n_src=40, nrhs=nrhs, seed=9)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail)
    s.factorize(dev(c.values))
    B = dev(c.rhs)              # [nrhs, n]: column r at r*n
    X = torch.zeros_like(B)
    s.solve(B, X, nrhs=nrhs)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    a0 = s.analysis()
    lu = oracle_refactor(oracle_mod, c, c.values, a0, EPS, a0["pivrow"])
    kap = kappa_est(oracle_mod, lu, c, c.values, a0)
    for r in range(nrhs):
        eta = oracle_mod.backward_error(c.colptr, c.rowind, c.values, Xh[r], c.rhs[r])
        assert eta <= 1e-12
        xo = oracle_mod.solve(lu, a0["rowperm_pre"], a0["colperm"], c.rhs[r])
        eta_o = oracle_mod.backward_error(c.colptr, c.rowind, c.values, xo, c.rhs[r])
        check_solution(Xh[r], xo, kap, eta, eta_o, "rhs %d" % r)


@pytest.mark.parametrize("tail", [-1, 200])
def test_fp32_ir(ck, oracle_mod, tail):
    c = mnagen.mesh_transistor(50, 50, seed=12)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, precision=ck.CKTLU_FP32_IR, ir_tol=1e-10,
                    dense_tail=tail)
    s.factorize(dev(c.values))
    a0 = s.analysis()
    vh = mnagen.perturb(c.values, 12, 0, 1)
    lu = oracle_refactor(oracle_mod, c, vh, a0, EPS, a0["pivrow"])
    rc, info = s.refactorize(dev(vh))
    assert rc == (ck.CKTLU_W_REPIVOTED if lu.nswaps else 0)
    assert np.array_equal(s.analysis()["pivrow"], lu.pivrow)
    b = c.rhs[0]
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    rc, sinfo = s.solve(dev(b), x)
    torch.cuda.synchronize()
    xg = x.cpu().numpy()
    eta = oracle_mod.backward_error(c.colptr, c.rowind, vh, xg, b)
    assert eta <= 1e-10, (eta, sinfo.ir_iters, sinfo.used_fp64)
    # forward error against the FP64 oracle: at most about kappa(A) times the backward errors
    xo = oracle_mod.solve(lu, a0["rowperm_pre"], a0["colperm"], b)
    eta_o = oracle_mod.backward_error(c.colptr, c.rowind, vh, xo, b)
    kap = kappa_est(oracle_mod, lu, c, vh, a0)
    wx = check_solution(xg, xo, kap, eta, eta_o, "fp32+ir")
    say("fp32+ir eta %.2e iters %d x/tol %.2e kappa %.2e" % (eta, sinfo.ir_iters, wx, kap))
    # a second solve with the same factors (the dense block is re-read, not re-factored)
    x2 = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    s.solve(dev(b), x2)
    torch.cuda.synchronize()
    assert oracle_mod.backward_error(c.colptr, c.rowind, vh, x2.cpu().numpy(), b) <= 1e-10


@pytest.mark.parametrize("tail", [-1, 10 ** 6])
def test_tiny_and_degenerate(ck, oracle_mod, tail):
    for kind, n in [("diagonal", 1), ("diagonal", 7), ("dense", 12), ("tridiagonal", 200),
                    ("arrow_first", 40), ("permutation", 9), ("dense", 130)]:
        c = mnagen.hand_pattern(kind, n, seed=3)
        say("case", kind, n, "tail", tail)
        s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail)
        s.factorize(dev(c.values))
        vh = mnagen.perturb(c.values, 3, 0, 1)
        rc, info = s.refactorize(dev(vh))
        a = s.analysis()
        lu = oracle_refactor(oracle_mod, c, vh, a, EPS, a["pivrow"])
        compare_factors(s.factors(), lu)
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
        s.solve(dev(c.rhs[0]), x)
        torch.cuda.synchronize()
        eta = oracle_mod.backward_error(c.colptr, c.rowind, vh, x.cpu().numpy(), c.rhs[0])
        assert eta <= 1e-12, (kind, n, eta)


@pytest.mark.parametrize("tail", [-1, 100])
def test_batched_equals_single(ck, tail):
    c = mnagen.mesh_transistor(30, 30, seed=13)
    batch = 5
    V = mnagen.instance_values(c, batch, 0.3, seed=13)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail)
    s.factorize(dev(c.values))
    status = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
    s.refactorize_batched(batch, dev(V), status)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    single = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail)
    single.factorize(dev(c.values))
    for i in range(batch):
        fb = s.factors(instance=i)
        if st[i] != -1:
            continue
        rc, _ = single.refactorize(dev(V[i]))
        if rc != 0:
            continue
        fs = single.factors()
        assert np.array_equal(fb["Lx"], fs["Lx"]) and np.array_equal(fb["Ux"], fs["Ux"]), i
    assert (st == -1).sum() >= 1


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("tail", [-1, 100])
def test_solve_batched(ck, oracle_mod, tail, precision):
    """Batched solves after a batched refactorization: every instance that
    passed its check is solved to eta <= 1e-12 (FP64) or refined to <= 1e-10
    (FP32 factors, FP64 refinement per instance); failed instances are skipped."""
    c = mnagen.mesh_transistor(30, 30, seed=14)
    batch, nrhs = 4, 2
    V = mnagen.instance_values(c, batch, 0.2, seed=14)
    prec = ck.CKTLU_FP64 if precision == "fp64" else ck.CKTLU_FP32_IR
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail, precision=prec, ir_tol=1e-10)
    s.factorize(dev(c.values))
    status = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
    s.refactorize_batched(batch, dev(V), status)
    rng = np.random.default_rng(14)
    B = rng.standard_normal((batch, nrhs, c.n))
    X = torch.full((batch, nrhs, c.n), 7.0, dtype=torch.float64, device="cuda:0")
    eta_dev = torch.zeros(batch, dtype=torch.float64, device="cuda:0")
    rc = s.solve_batched(batch, nrhs, dev(B), X, status, eta_dev)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    Xh = X.cpu().numpy()
    eh = eta_dev.cpu().numpy()
    assert (st == -1).sum() >= 1
    tol = 1e-12 if precision == "fp64" else 1e-10
    for i in range(batch):
        if st[i] != -1:
            assert np.all(Xh[i] == 7.0)
            continue
        etas = [oracle_mod.backward_error(c.colptr, c.rowind, V[i], Xh[i, r], B[i, r]) for r in range(nrhs)]
        assert max(etas) <= tol, (i, etas)
        if precision == "fp32_ir":
            assert 0 <= eh[i] <= 1e-10 and abs(eh[i] - max(etas)) <= 0.05 * max(etas) + 1e-15, (eh[i], etas)
        else:
            assert eh[i] == -1.0
    if precision == "fp32_ir":
        assert rc in (0, ck.CKTLU_W_IR_FALLBACK)


def test_batched_many_instances_dense_block(ck, oracle_mod):
    """64 instances with a four-panel dense block: the panels of different
    instances run in one launch, so no instance may see another stage of its
    own diagonal block than the one its panel factors; every instance equals
    its single refactorization bit for bit and solves to eta <= 1e-12."""
    c = mnagen.mesh_transistor(30, 30, seed=15)
    batch, tail = 64, 256
    V = mnagen.instance_values(c, batch, 0.3, seed=15)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail)
    s.factorize(dev(c.values))
    status = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
    s.refactorize_batched(batch, dev(V), status)
    B = np.repeat(c.rhs[:1][None], batch, axis=0)
    X = torch.zeros((batch, 1, c.n), dtype=torch.float64, device="cuda:0")
    s.solve_batched(batch, 1, dev(B), X, status)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    Xh = X.cpu().numpy()
    single = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail)
    single.factorize(dev(c.values))
    checked = 0
    for i in range(batch):
        if st[i] != -1:
            continue
        assert oracle_mod.backward_error(c.colptr, c.rowind, V[i], Xh[i, 0], B[i, 0]) <= 1e-12, i
        if i % 8 == 7:
            rc, _ = single.refactorize(dev(V[i]))
            if rc == 0:
                fb, fs = s.factors(instance=i), single.factors()
                assert np.array_equal(fb["Lx"], fs["Lx"]) and np.array_equal(fb["Ux"], fs["Ux"]), i
                checked += 1
    assert checked >= 4


def test_fp32_ir_fallback_then_fp64(ck, oracle_mod):
    """Refinement that cannot reach its target (ir_tol below FP64 rounding) falls
    back to FP64 factors (W_IR_FALLBACK); the context then stays on FP64 factors
    for the next steps, whose solves meet the FP64 gate, until factorize."""
    c = mnagen.mesh_transistor(40, 40, seed=18)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, precision=ck.CKTLU_FP32_IR, ir_tol=1e-30, ir_max_iter=3)
    s.factorize(dev(c.values))
    b = c.rhs[0]
    for t in (1, 2):
        v = mnagen.restamp(c, 18, 0, t)
        s.refactorize(dev(v))
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
        rc, info = s.solve(dev(b), x)
        torch.cuda.synchronize()
        assert info.used_fp64 == 1
        assert rc == (ck.CKTLU_W_IR_FALLBACK if t == 1 else 0)
        assert oracle_mod.backward_error(c.colptr, c.rowind, v, x.cpu().numpy(), b) <= 1e-12
    assert s.stats()["n_fp64_fallback_solves"] == 1
    s.factorize(dev(c.values))                     # back to FP32 factors
    s.refactorize(dev(c.values))
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    rc, info = s.solve(dev(b), x)
    assert info.used_fp64 == 1 and rc == ck.CKTLU_W_IR_FALLBACK   # the target is still out of reach


@pytest.mark.parametrize("width", [0, -1])
def test_fp32_check_retry_keeps_fp64(ck, oracle_mod, width):
    """A pivot exactly at the threshold in FP64 (|a| = eps |c|) that rounds below it in FP32:
    the FP32 refactorization fails its test, the FP64 retry passes (no re-pivot, the oracle's
    pivots), and the context then keeps FP64 factors for its solves and later steps until
    the next factorize."""
    import struct
    eps = 0.00099999996                    # float32(eps) rounds down, below eps
    assert struct.unpack("f", struct.pack("f", eps))[0] < eps
    colptr = np.array([0, 2, 4], np.int32)
    rowind = np.array([0, 1, 0, 1], np.int32)
    vals = np.array([eps, 1.0, 1.0, 3.0])   # A = [[eps, 1], [1, 3]]
    b = np.array([1.0, 2.0])
    s = ck.SparseLU(2, colptr, rowind, eps=eps, precision=ck.CKTLU_FP32_IR, ordering=ck.CKTLU_ORDER_NATURAL,
                    dense_tail=-1, sweep_supernodes=width)
    s.factorize(dev(vals))
    assert list(s.analysis()["pivrow"]) == [0, 1]
    for step in range(2):
        rc, info = s.refactorize(dev(vals))
        assert rc == 0 and info.repivoted == 0
        assert list(s.analysis()["pivrow"]) == [0, 1]
        x = torch.zeros(2, dtype=torch.float64, device="cuda:0")
        rc, sinfo = s.solve(dev(b), x)
        torch.cuda.synchronize()
        assert rc == 0 and sinfo.used_fp64 == 1
        assert oracle_mod.backward_error(colptr, rowind, vals, x.cpu().numpy(), b) <= 1e-12
    assert s.stats()["n_fp32_check_retries"] == 1
    s.factorize(dev(vals))                  # back to FP32 factors: the retry happens again
    s.refactorize(dev(vals))
    assert s.stats()["n_fp32_check_retries"] == 2


@pytest.mark.parametrize("tail", [-1, 100])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_solve_chain_widths_identical(ck, oracle_mod, tail, nrhs):
    """Chained solve launches (runs of narrow levels in one workgroup per
    instance) compute every row exactly as the per-level launches do, so the
    solutions are bit-identical for any chain width: -1 (no chains), 0 (the
    default), 8 (short chains) and 10**9 (every level, the dense rows' level
    included, chained); batched instances with one skipped instance too."""
    c = mnagen.layered_rc(24, 24, 3, seed=21)
    batch = 3
    V = mnagen.instance_values(c, batch, 0.05, seed=21)
    rng = np.random.default_rng(21)
    B = rng.standard_normal((batch, nrhs, c.n))
    B1 = rng.standard_normal((nrhs, c.n))
    outs = {}
    for w in (-1, 0, 8, 10 ** 9):
        say("chain width", w, "tail", tail, "nrhs", nrhs)
        s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail, solve_chain_width=w)
        s.factorize(dev(c.values))
        X = torch.zeros((nrhs, c.n), dtype=torch.float64, device="cuda:0")
        s.solve(dev(B1), X, nrhs=nrhs)
        status = torch.tensor([-1, 5, -1], dtype=torch.int32, device="cuda:0")
        Xb = torch.full((batch, nrhs, c.n), 7.0, dtype=torch.float64, device="cuda:0")
        s.refactorize_batched(batch, dev(V), torch.zeros(batch, dtype=torch.int32, device="cuda:0"))
        s.solve_batched(batch, nrhs, dev(B), Xb, status)
        torch.cuda.synchronize()
        outs[w] = (X.cpu().numpy(), Xb.cpu().numpy())
    for w in (0, 8, 10 ** 9):
        assert np.array_equal(outs[w][0], outs[-1][0]), w
        assert np.array_equal(outs[w][1], outs[-1][1]), w
    X, Xb = outs[0]
    for r in range(nrhs):
        assert oracle_mod.backward_error(c.colptr, c.rowind, c.values, X[r], B1[r]) <= 1e-12
    assert np.all(Xb[1] == 7.0)
    for i in (0, 2):
        for r in range(nrhs):
            assert oracle_mod.backward_error(c.colptr, c.rowind, V[i], Xb[i, r], B[i, r]) <= 1e-12


@pytest.mark.parametrize("width", [64, 128, 256])
@pytest.mark.parametrize("tail", [300, 520])
def test_dense_panel_widths(ck, oracle_mod, width, tail):
    """Groups of 64, 128 or 256 dense columns between updates of the whole trailing
    block (full groups, a ragged last group, a ragged last panel): factors match
    the oracle's, the solve reaches eta <= 1e-12, and a batch of instances gives
    every instance's factors of the single-instance path."""
    c = mnagen.mesh_transistor(40, 40, seed=23)
    say("dense panel width", width, "tail", tail)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail, dense_panel_width=width)
    s.factorize(dev(c.values))
    a0 = s.analysis()
    vh = mnagen.restamp(c, 23, 0, 1)
    rc, info = s.refactorize(dev(vh))
    lu = oracle_refactor(oracle_mod, c, vh, a0, EPS, a0["pivrow"])
    assert np.array_equal(s.analysis()["pivrow"], lu.pivrow)
    f1 = s.factors()
    compare_factors(f1, lu)
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    s.solve(dev(c.rhs[0]), x)
    torch.cuda.synchronize()
    assert oracle_mod.backward_error(c.colptr, c.rowind, vh, x.cpu().numpy(), c.rhs[0]) <= 1e-12
    if rc == 0:
        batch = 3
        V = np.stack([vh, mnagen.restamp(c, 23, 0, 2), vh])
        st = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
        s.refactorize_batched(batch, dev(V), st)
        torch.cuda.synchronize()
        assert st.cpu().numpy()[0] == -1 and st.cpu().numpy()[2] == -1
        for i in (0, 2):
            fb = s.factors(instance=i)
            for k in ("Lx", "Ux"):
                assert np.array_equal(fb[k], f1[k]), (i, k)


@pytest.mark.parametrize("width", [64, 256])
def test_dense_lookahead_identical(ck, width):
    """The look-ahead (the next group's panels on a second stream while the trailing
    update of the current group runs) performs the same operations on disjoint parts of
    the dense block, so factors and solutions are bit-identical to one stream; a
    batch of instances with one failing sweep included."""
    c = mnagen.mesh_transistor(40, 40, seed=24)
    batch = 3
    V = mnagen.instance_values(c, batch, 0.1, seed=24)
    out = {}
    for la in (0, 1):
        say("lookahead", la, "width", width)
        s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=600, dense_panel_width=width,
                        dense_lookahead=la)
        s.factorize(dev(c.values))
        st = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
        s.refactorize_batched(batch, dev(V), st)
        X = torch.zeros((batch, 1, c.n), dtype=torch.float64, device="cuda:0")
        s.solve_batched(batch, 1, dev(np.repeat(c.rhs[:1][None], batch, axis=0)), X, st)
        torch.cuda.synchronize()
        out[la] = ([s.factors(instance=i) for i in range(batch)], X.cpu().numpy(), st.cpu().numpy())
    assert np.array_equal(out[0][2], out[1][2])
    assert np.array_equal(out[0][1], out[1][1])
    for i in range(batch):
        for k in ("Lx", "Ux"):
            assert np.array_equal(out[0][0][i][k], out[1][0][i][k]), (i, k)


SLOT_MAP_CASES = [
    ("mesh_transistor_40", lambda: mnagen.mesh_transistor(40, 40, seed=31), 600),
    ("random_1400", lambda: mnagen.random_pattern(1400, 0.01, 8), -1),         # no dense block; columns > 1024 rows
]


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("name,make,tail", SLOT_MAP_CASES, ids=[s[0] for s in SLOT_MAP_CASES])
def test_slot_map_identical(ck, name, make, tail, precision):
    """The sweep's slot map replaces the search of the target rows by a load of the
    slot; the updates and their order are the same, so factors, solutions and statuses
    are bit-identical to the search path, single and batched (one instance failing its
    pivot check)."""
    c = make()
    batch = 3
    V = np.stack([mnagen.perturb(c.values, 31, 0, t) for t in range(batch)])
    prec = ck.CKTLU_FP64 if precision == "fp64" else ck.CKTLU_FP32_IR
    h = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail)
    h.factorize_host(c.values)
    lev, nl = h.levels(), np.diff(h.factors()["Lp"])
    kf = [k for k in range(c.n) if lev[k] == 1 and nl[k] > 0][0]
    V[1, _pivot_entry(c, h.analysis(), kf)] *= 1e-8       # instance 1 fails its pivot check
    out = {}
    for m in (-1, 0):
        say(name, precision, "slot map", m)
        s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail, sweep_slot_map=m, precision=prec,
                        sweep_supernodes=-1)                   # the slot map belongs to the column sweep
        s.factorize(dev(c.values))
        assert (s.stats()["slot_map_entries"] > 0) == (m == 0)
        s.refactorize(dev(V[0]))
        f1 = s.factors()
        st = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
        s.refactorize_batched(batch, dev(V), st)
        X = torch.zeros((batch, 1, c.n), dtype=torch.float64, device="cuda:0")
        s.solve_batched(batch, 1, dev(np.repeat(c.rhs[:1][None], batch, axis=0)), X, st)
        torch.cuda.synchronize()
        out[m] = (f1, [s.factors(instance=i) for i in (0, 2)], X.cpu().numpy(), st.cpu().numpy())
    assert np.array_equal(out[-1][3], out[0][3])
    assert 0 <= out[0][3][1] <= kf and out[0][3][0] == -1 and out[0][3][2] == -1
    assert np.array_equal(out[-1][2][[0, 2]], out[0][2][[0, 2]])
    for k in ("Lx", "Ux"):
        assert np.array_equal(out[-1][0][k], out[0][0][k]), k
        for i in range(2):
            assert np.array_equal(out[-1][1][i][k], out[0][1][i][k]), (i, k)


LONG_ROWS = [
    ("power_grid_80", lambda: mnagen.power_grid(80, 80, n_src=50, seed=3)),      # L rows up to ~330
    ("random_700", lambda: mnagen.random_pattern(700, 0.01, 6)),                 # L and U rows > 256
    ("random_1400", lambda: mnagen.random_pattern(1400, 0.01, 8)),               # L rows > 1024 (two passes)
]


@pytest.mark.parametrize("nrhs", [1, 3])
@pytest.mark.parametrize("name,make", LONG_ROWS, ids=[s[0] for s in LONG_ROWS])
def test_solve_long_rows(ck, oracle_mod, name, make, nrhs):
    """Levels holding a row longer than 64 entries run a workgroup per row (rows past
    1024 entries take several passes); the solutions reach eta <= 1e-12 and agree
    with the oracle's, single and batched (one skipped instance), FP64 and FP32
    factors with refinement."""
    c = make()
    say("long rows", name, "n", c.n, "nrhs", nrhs)
    rng = np.random.default_rng(31)
    B = rng.standard_normal((nrhs, c.n))
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=-1)
    s.factorize(dev(c.values))
    a0 = s.analysis()
    X = torch.zeros((nrhs, c.n), dtype=torch.float64, device="cuda:0")
    s.solve(dev(B), X, nrhs=nrhs)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    lu = oracle_refactor(oracle_mod, c, c.values, a0, EPS, a0["pivrow"])
    kap = kappa_est(oracle_mod, lu, c, c.values, a0)
    for r in range(nrhs):
        eta = oracle_mod.backward_error(c.colptr, c.rowind, c.values, Xh[r], B[r])
        assert eta <= 1e-12
        xo = oracle_mod.solve(lu, a0["rowperm_pre"], a0["colperm"], B[r])
        eta_o = oracle_mod.backward_error(c.colptr, c.rowind, c.values, xo, B[r])
        check_solution(Xh[r], xo, kap, eta, eta_o, "%s rhs %d" % (name, r))
    batch = 3
    V = np.stack([mnagen.perturb(c.values, 31, 0, i) for i in range(batch)])
    for prec, tol in ((ck.CKTLU_FP64, 1e-12), (ck.CKTLU_FP32_IR, 1e-10)):
        sb = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=-1, precision=prec, ir_tol=1e-10)
        sb.factorize(dev(c.values))
        st = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
        sb.refactorize_batched(batch, dev(V), st)
        st = torch.tensor(np.where(np.arange(batch) == 1, 4, st.cpu().numpy()), dtype=torch.int32, device="cuda:0")
        Bb = rng.standard_normal((batch, nrhs, c.n))
        Xb = torch.full((batch, nrhs, c.n), 7.0, dtype=torch.float64, device="cuda:0")
        sb.solve_batched(batch, nrhs, dev(Bb), Xb, st)
        torch.cuda.synchronize()
        Xbh = Xb.cpu().numpy()
        sth = st.cpu().numpy()
        assert np.all(Xbh[1] == 7.0)
        for i in (0, 2):
            if sth[i] != -1:
                continue
            for r in range(nrhs):
                assert oracle_mod.backward_error(c.colptr, c.rowind, V[i], Xbh[i, r], Bb[i, r]) <= tol, (prec, i, r)


def test_restart_set_deterministic(ck, oracle_mod):
    """Pivots of several columns made to fail in one refactorization: the set of
    unfinished columns the device leaves is the same in repeated runs (the interrupt
    word records the failing level, so no wavefront's timing decides it), it holds
    the first failing column, and the restart set is the oracle's closure of it on
    the library's elimination tree (Section IV-C); restart_size counts it."""
    c = mnagen.mesh_transistor(30, 30, seed=25)
    h = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=100)
    h.factorize_host(c.values)
    a0, lev, nl = h.analysis(), h.levels(), np.diff(h.factors()["Lp"])
    cand = [k for k in range(c.n - 100) if lev[k] <= 1 and nl[k] > 0]
    chosen = cand[::max(1, len(cand) // 6)][:6]
    vh = mnagen.perturb(c.values, 25, 0, 1)
    for k in chosen:
        vh[_pivot_entry(c, a0, k)] *= 1e-8
    runs = []
    for rep in range(3):
        s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=100)
        s.factorize(dev(c.values))
        rc, info = s.refactorize(dev(vh))
        assert rc == ck.CKTLU_W_REPIVOTED
        unf, rs = s.last_restart()
        runs.append((info.first_fail_col, unf, rs, info.restart_size))
        s.close()
    for r in runs[1:]:
        assert r[0] == runs[0][0]
        assert np.array_equal(r[1], runs[0][1]) and np.array_equal(r[2], runs[0][2])
    first, unf, rs, size = runs[0]
    assert first in chosen and unf[first]
    assert np.array_equal(rs, oracle_mod.restart_set(a0["parent"], unf))
    assert size == int(rs.sum())


def test_factorize_host_then_fp32_ir_solve(ck, oracle_mod):
    """factorize_host followed directly by an FP32_IR solve: the refinement's
    residual uses the factorized values (uploaded with the factors), so x equals the
    oracle's solution of that matrix within the kappa-scaled bound."""
    c = mnagen.mesh_transistor(30, 30, seed=26)
    vh = mnagen.restamp(c, 26, 0, 3)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, precision=ck.CKTLU_FP32_IR, ir_tol=1e-10)
    s.factorize_host(vh)
    b = c.rhs[0]
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    rc, info = s.solve(dev(b), x)
    torch.cuda.synchronize()
    xg = x.cpu().numpy()
    eta = oracle_mod.backward_error(c.colptr, c.rowind, vh, xg, b)
    assert rc == 0 and info.used_fp64 == 0 and eta <= 1e-10, (rc, info.used_fp64, eta)
    a0 = s.analysis()
    lu = oracle_refactor(oracle_mod, c, vh, a0, EPS, np.arange(c.n))
    assert lu.status == 0 and np.array_equal(lu.pivrow, a0["pivrow"])
    xo = oracle_mod.solve(lu, a0["rowperm_pre"], a0["colperm"], b)
    eta_o = oracle_mod.backward_error(c.colptr, c.rowind, vh, xo, b)
    check_solution(xg, xo, kappa_est(oracle_mod, lu, c, vh, a0), eta, eta_o, "factorize_host + fp32_ir")


SN_CASES = [
    ("mesh_transistor_40", lambda: mnagen.mesh_transistor(40, 40, seed=41)),
    ("layered_rc_3x24", lambda: mnagen.layered_rc(24, 24, 3, seed=42)),
    ("power_grid_60", lambda: mnagen.power_grid(60, 60, n_src=50, seed=43)),
    ("random_300", lambda: mnagen.random_pattern(300, 0.01, 44)),
]


@pytest.mark.parametrize("tail", [-1, 100])
@pytest.mark.parametrize("width", [-1, 8, 0])
@pytest.mark.parametrize("name,make", SN_CASES, ids=[c[0] for c in SN_CASES])
def test_supernodal_sweep_vs_oracle(ck, oracle_mod, name, make, width, tail):
    """The sweep on supernodes of at most 8 or 64 columns (and the column sweep, -1): pattern
    and pivots bit-exact, values within the per-entry rounding bound, reconstruction within
    GE's backward error; FP32 factors refine to eta <= 1e-10; a batch of instances gives
    each instance's single factors bit for bit."""
    c = make()
    say("supernodal", name, "width", width, "tail", tail)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail, sweep_supernodes=width)
    s.factorize(dev(c.values))
    a0 = s.analysis()
    st = s.stats()
    assert (st["sweep_supernodes"] > 0) == (width >= 0 and st["n"] > (st["dense_tail"] or 0))
    vh = mnagen.restamp(c, 41, 0, 1)
    rc, info = s.refactorize(dev(vh))
    lu = oracle_refactor(oracle_mod, c, vh, a0, EPS, a0["pivrow"])
    assert np.array_equal(s.analysis()["pivrow"], lu.pivrow)
    f = s.factors()
    w = compare_factors(f, lu)
    wb = check_backward_factors(f, c, vh, a0, lu.pivrow)
    say("  levels", st["sweep_levels"], "supernodes", st["sweep_supernodes"], "factor/tol %.2e backward/tol %.2e" % (w, wb))
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    s.solve(dev(c.rhs[0]), x)
    torch.cuda.synchronize()
    assert oracle_mod.backward_error(c.colptr, c.rowind, vh, x.cpu().numpy(), c.rhs[0]) <= 1e-12
    if rc == 0:
        batch = 3
        V = np.stack([vh, mnagen.restamp(c, 41, 0, 2), vh])
        stt = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
        s.refactorize_batched(batch, dev(V), stt)
        torch.cuda.synchronize()
        if stt.cpu().numpy()[2] == -1:
            fb = s.factors(instance=2)
            assert np.array_equal(fb["Lx"], f["Lx"]) and np.array_equal(fb["Ux"], f["Ux"])
    s32 = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail, sweep_supernodes=width,
                      precision=ck.CKTLU_FP32_IR, ir_tol=1e-10)
    s32.factorize(dev(c.values))
    s32.refactorize(dev(vh))
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    s32.solve(dev(c.rhs[0]), x)
    torch.cuda.synchronize()
    assert oracle_mod.backward_error(c.colptr, c.rowind, vh, x.cpu().numpy(), c.rhs[0]) <= 1e-10


@pytest.mark.parametrize("tail", [-1, 100])
@pytest.mark.parametrize("name,make", SN_CASES, ids=[c[0] for c in SN_CASES])
def test_supernodal_split_units_vs_oracle(ck, oracle_mod, name, make, tail):
    """Panels split into units of 16 rows (8 for panels of at most 16 columns) and supernodal
    solves split into units of four runs (solve_split_entries = 64), so that the arrival counters and the slice
    combines run on small circuits: the factors equal those of the unsplit schedule bit for
    bit (splitting rows of R changes no operation), pattern and pivots equal the oracle's,
    the solutions reach eta <= 1e-12 (FP64; 1e-10 refined from FP32 factors, one and eight
    right-hand sides, a batch of three instances) and agree with the oracle's within the
    condition-scaled bound; the test is repeated to catch counters not reset."""
    c = make()
    say("split units", name, "tail", tail)
    vh = mnagen.restamp(c, 47, 0, 1)
    ref = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail)
    ref.factorize(dev(c.values))
    a0 = ref.analysis()
    ref.refactorize(dev(vh))
    fref = ref.factors()
    lu = oracle_refactor(oracle_mod, c, vh, a0, EPS, a0["pivrow"])
    kap = kappa_est(oracle_mod, lu, c, vh, a0)
    for prec in (ck.CKTLU_FP64, ck.CKTLU_FP32_IR):
        s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail, precision=prec, ir_tol=1e-10,
                        sweep_panel_rows=16, solve_split_entries=64)
        s.factorize(dev(c.values))
        for rep in range(2):
            rc, info = s.refactorize(dev(vh))
            assert np.array_equal(s.analysis()["pivrow"], lu.pivrow)
            if prec == ck.CKTLU_FP64:
                f = s.factors()
                for key in ("Lp", "Li", "Lx", "Up", "Ui", "Ux"):
                    assert np.array_equal(f[key], fref[key]), key
            for nrhs in (1, 8):
                B = np.stack([c.rhs[r % len(c.rhs)] * (1.0 + r) for r in range(nrhs)])
                X = torch.zeros((nrhs, c.n), dtype=torch.float64, device="cuda:0")
                s.solve(dev(B), X, nrhs=nrhs)
                torch.cuda.synchronize()
                Xh = X.cpu().numpy()
                tol = 1e-12 if prec == ck.CKTLU_FP64 else 1e-10
                for r in range(nrhs):
                    eta = oracle_mod.backward_error(c.colptr, c.rowind, vh, Xh[r], B[r])
                    assert eta <= tol, (nrhs, r, eta)
                    xo = oracle_mod.solve(lu, a0["rowperm_pre"], a0["colperm"], B[r])
                    eta_o = oracle_mod.backward_error(c.colptr, c.rowind, vh, xo, B[r])
                    check_solution(Xh[r], xo, kap, eta, eta_o, "split rhs %d/%d" % (r, nrhs))
        if rc == 0:
            batch = 3
            V = np.stack([vh, mnagen.restamp(c, 47, 0, 2), vh])
            stt = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
            s.refactorize_batched(batch, dev(V), stt)
            B = np.stack([c.rhs[0]] * batch)
            X = torch.zeros((batch, c.n), dtype=torch.float64, device="cuda:0")
            eta_d = torch.zeros(batch, dtype=torch.float64, device="cuda:0")
            s.solve_batched(batch, 1, dev(B), X, stt, eta_d)
            torch.cuda.synchronize()
            st_h = stt.cpu().numpy()
            for i in range(batch):
                if st_h[i] == -1:
                    vi = V[i]
                    eta = oracle_mod.backward_error(c.colptr, c.rowind, vi, X[i].cpu().numpy(), B[i])
                    assert eta <= (1e-12 if prec == ck.CKTLU_FP64 else 1e-10), (i, eta)


def test_supernodal_panel_failure_fallback(ck, oracle_mod):
    """The pivot test forced to fail at a column inside a wide supernode (a panel): the
    fallback's result equals the oracle's re-factorization, and the unfinished set holds
    the failing column."""
    c = mnagen.power_grid(60, 60, n_src=50, seed=45)
    h = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=-1)
    h.factorize_host(c.values)
    f0 = h.factors()
    # a column whose L pattern continues its predecessor's (inside a supernode), well inside
    Lp, Li = f0["Lp"], f0["Li"]
    col = None
    for k in range(c.n // 2, c.n - 2):
        if Lp[k] < Lp[k + 1] and Li[Lp[k]] == k + 1 and Lp[k + 1] - Lp[k] == Lp[k + 2] - Lp[k + 1] + 1:
            col = k + 1
            break
    assert col is not None
    o = ck.cktlu_default_options()
    o.pivot_eps = EPS
    o.force_fail_col = col
    o.dense_tail_size = -1
    ctx = ck.cktlu_create(o)
    try:
        assert ck.cktlu_analyze(ctx, c.n, c.colptr, c.rowind) == 0
        assert ck.cktlu_factorize(ctx, dev(c.values)) == 0
        n = c.n
        rp, cp, pv, par = (np.zeros(n, np.int32) for _ in range(4))
        assert ck.cktlu_get_analysis(ctx, rp, cp, pv, par) == 0
        vh = mnagen.restamp(c, 45, 0, 1)
        info = ck.cktlu_refactor_info()
        rc = ck.cktlu_refactorize(ctx, dev(vh), info)
        assert rc == ck.CKTLU_W_REPIVOTED and info.first_fail_col == col
        unf, rs = np.zeros(n, np.int32), np.zeros(n, np.int32)
        assert ck.cktlu_get_last_restart(ctx, unf, rs) == 0
        assert unf[col] == 1 and rs[col] == 1
        assert np.array_equal(rs.astype(bool), oracle_mod.restart_set(par, unf.astype(bool)))
        lu = oracle_refactor(oracle_mod, c, vh, dict(rowperm_pre=rp, colperm=cp), EPS, pv)
        pv2 = np.zeros(n, np.int32)
        assert ck.cktlu_get_analysis(ctx, None, None, pv2, None) == 0
        assert np.array_equal(pv2, lu.pivrow)
    finally:
        ck.cktlu_destroy(ctx)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_static_pivoting_scaling_gpu(ck, oracle_mod, precision):
    """Pre-processing with values (maximum-product matching and scaling, Section III-A): the
    device refactorization factors S_r P A S_c, equal to the oracle's factorization of that
    matrix; solutions solve the caller's unscaled system (eta <= 1e-12, 1e-10 with FP32
    factors and refinement) and a batch gives each instance's single factors bit for bit."""
    c = mnagen.mesh_vsrc(24, 24, 4, seed=61)
    prec = ck.CKTLU_FP64 if precision == "fp64" else ck.CKTLU_FP32_IR
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, static_pivoting=2, values=c.values, precision=prec,
                    ir_tol=1e-10, dense_tail=100)
    s.factorize(dev(c.values))
    a0 = s.analysis()
    rs, cs = s.scaling()
    assert not np.all(rs == 1.0)
    cols = np.repeat(np.arange(c.n), np.diff(c.colptr))
    vh = mnagen.restamp(c, 61, 0, 1)
    rc, info = s.refactorize(dev(vh))
    vs = vh * rs[c.rowind] * cs[cols]
    lu = oracle_refactor(oracle_mod, c, vs, a0, EPS, a0["pivrow"])
    assert lu.status == 0 and np.array_equal(s.analysis()["pivrow"], lu.pivrow)
    if precision == "fp64":
        compare_factors(s.factors(), lu)
    b = c.rhs[0]
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    s.solve(dev(b), x)
    torch.cuda.synchronize()
    eta = oracle_mod.backward_error(c.colptr, c.rowind, vh, x.cpu().numpy(), b)
    assert eta <= (1e-12 if precision == "fp64" else 1e-10), eta
    if precision == "fp64":
        batch = 3
        V = np.stack([vh, mnagen.restamp(c, 61, 0, 2), vh])
        st = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
        s.refactorize_batched(batch, dev(V), st)
        X = torch.zeros((batch, 1, c.n), dtype=torch.float64, device="cuda:0")
        s.solve_batched(batch, 1, dev(np.repeat(c.rhs[:1][None], batch, axis=0)), X, st)
        torch.cuda.synchronize()
        sth, Xh = st.cpu().numpy(), X.cpu().numpy()
        for i in range(batch):
            if sth[i] == -1:
                assert oracle_mod.backward_error(c.colptr, c.rowind, V[i], Xh[i, 0], b) <= 1e-12
        if sth[2] == -1:
            fb = s.factors(instance=2)
            f1 = s.factors()
            assert np.array_equal(fb["Lx"], f1["Lx"])
