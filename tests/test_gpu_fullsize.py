"""GPU parity at the full sizes of the workloads (the launch configuration of bench.py).

- Post-layout RC mesh 3 x 300 x 300 (n = 270,000; the benchmark workload):
  refactorizations with re-stamped values, pattern and pivot sequence bit-exact
  against the oracle's re-factorization, values on sampled entries within the
  |L||U| rounding scale, eta_inf <= 1e-12 (FP64) and <= 1e-10 (FP32 + IR).
- 256 same-pattern corners of a 141 x 141 mesh with transistor stamps
  (n = 19,881, per-element log-normal values, sigma = 0.3) in one batched
  refactorization: every instance's solve reaches its gate (FP64 and FP32 + IR),
  sampled instances equal their single refactorization bit for bit and the
  oracle within rounding.
- 1000 x 1000 power grid (n = 1,000,000) with 8 right-hand sides: the FP64
  refactorization's pattern and pivot sequence bit-exact against the oracle's,
  sampled values within rounding, every right-hand side's solution within the
  condition-scaled bound of the oracle's; then FP32 factors with FP64 refinement,
  eta_inf <= 1e-10 and the same forward bound for every right-hand side.
- The RC mesh with a pivot inside its dense block made to fail: the dense block
  is re-factored on the device with the threshold pivot rule, and pattern and
  pivot sequence equal the oracle's re-factorization, values within rounding.
"""
import sys
import time

import numpy as np
import pytest
import scipy.sparse as sp

import mnagen
from helpers import (check_solution, compare_factors, compare_factors_sampled, kappa_est, oracle_refactor,
                     pivot_entry)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = 1e-3


@pytest.fixture(scope="module")
def ck():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_14082_amd as m
    return m


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda:0")


def say(t0, *a):
    print("[%6.1fs]" % (time.time() - t0), *a, flush=True)
    sys.stdout.flush()


def eta_inf(c, values, x, b):
    A = sp.csc_matrix((values, c.rowind, c.colptr), shape=(c.n, c.n))
    r = b - A @ x
    return float(np.abs(r).max() / (abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max()))


@pytest.mark.timeout(600)
def test_rc_mesh_3x300_full(ck, oracle_mod):
    t0 = time.time()
    c = mnagen.layered_rc(300, 300, 3, seed=0)
    say(t0, "layered_rc_3x300 n", c.n, "nnz", c.nnz)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS)
    s.factorize(dev(c.values))
    a0 = s.analysis()
    say(t0, "factorized; dense tail", s.stats()["dense_tail"])
    b = c.rhs[0]
    for t in (1, 2):
        v = mnagen.restamp(c, 0, 2, t)
        rc, info = s.refactorize(dev(v))
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
        s.solve(dev(b), x)
        torch.cuda.synchronize()
        e = eta_inf(c, v, x.cpu().numpy(), b)
        say(t0, "step", t, "rc", rc, "eta", e)
        assert e <= 1e-12
    lu = oracle_refactor(oracle_mod, c, v, a0, EPS, a0["pivrow"])
    say(t0, "oracle re-factorization done, swaps", lu.nswaps)
    assert lu.status == 0
    assert np.array_equal(s.analysis()["pivrow"], lu.pivrow)
    worst = compare_factors_sampled(s.factors(), lu)
    say(t0, "sampled scaled error", worst)
    s.close()
    # FP32 factors + FP64 refinement on the same values
    s32 = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, precision=ck.CKTLU_FP32_IR, ir_tol=1e-10)
    s32.factorize(dev(c.values))
    s32.refactorize(dev(v))
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    rc, sinfo = s32.solve(dev(b), x)
    torch.cuda.synchronize()
    e = eta_inf(c, v, x.cpu().numpy(), b)
    say(t0, "fp32+ir rc", rc, "iters", sinfo.ir_iters, "eta", e)
    assert e <= 1e-10
    # forward error against the FP64 oracle within the condition-scaled bound
    xo = oracle_mod.solve(lu, a0["rowperm_pre"], a0["colperm"], b)
    eta_o = eta_inf(c, v, xo, b)
    kap = kappa_est(oracle_mod, lu, c, v, a0)
    w = check_solution(x.cpu().numpy(), xo, kap, e, eta_o, "fp32+ir")
    say(t0, "fp32+ir forward difference / bound %.3e, kappa %.3e" % (w, kap))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("device", [0, -1], ids=["device", "host"])
def test_rc_mesh_3x300_dense_repivot_full(ck, oracle_mod, device):
    t0 = time.time()
    c = mnagen.layered_rc(300, 300, 3, seed=0)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_device_repivot=device)
    s.factorize(dev(c.values))
    a0 = s.analysis()
    D = s.stats()["dense_tail"]
    say(t0, "factorized; dense tail", D)
    v = mnagen.restamp(c, 0, 2, 1)
    lu1 = oracle_refactor(oracle_mod, c, v, a0, EPS, a0["pivrow"])
    assert lu1.status == 0 and lu1.nswaps == 0
    k = c.n - D + 1000                                # a column of the block's 16th panel
    assert lu1.Ui[lu1.Up[k + 1] - 1] == k
    v[pivot_entry(c, a0, k)] -= lu1.Ux[lu1.Up[k + 1] - 1] * (1 - 1e-8)
    lu = oracle_refactor(oracle_mod, c, v, a0, EPS, a0["pivrow"])
    say(t0, "oracle re-factorizations done, swaps", lu.nswaps)
    assert lu.status == 0 and lu.nswaps >= 1
    torch.cuda.synchronize()
    t1 = time.time()
    rc, info = s.refactorize(dev(v))
    torch.cuda.synchronize()
    say(t0, "refactorize with the dense re-pivot: %.2f s" % (time.time() - t1), "rc", rc)
    assert rc == ck.CKTLU_W_REPIVOTED and info.first_fail_col == k
    assert s.stats()["n_device_repivot"] == (1 if device == 0 else 0)
    assert np.array_equal(s.analysis()["pivrow"], lu.pivrow)
    worst = compare_factors_sampled(s.factors(), lu)
    say(t0, "sampled scaled error", worst)
    b = c.rhs[0]
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    s.solve(dev(b), x)
    torch.cuda.synchronize()
    assert eta_inf(c, v, x.cpu().numpy(), b) <= 1e-12
    rc, info = s.refactorize(dev(v))                   # the new pivot sequence now passes its check
    assert rc == 0 and info.repivoted == 0


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_batched_corners_256_full(ck, oracle_mod, precision):
    t0 = time.time()
    c = mnagen.mesh_transistor(141, 141, seed=0)
    batch = 256
    V = mnagen.instance_values(c, batch, 0.3, seed=3)
    prec = ck.CKTLU_FP64 if precision == "fp64" else ck.CKTLU_FP32_IR
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, precision=prec, ir_tol=1e-10)
    s.factorize(dev(c.values))
    a0 = s.analysis()
    say(t0, precision, "n", c.n, "batch", batch, "dense tail", s.stats()["dense_tail"])
    status = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
    Vd = dev(V)
    s.refactorize_batched(batch, Vd, status)
    B = np.repeat(c.rhs[:1][None, :, :], batch, axis=0)
    X = torch.zeros((batch, 1, c.n), dtype=torch.float64, device="cuda:0")
    s.solve_batched(batch, 1, dev(B), X, status)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    Xh = X.cpu().numpy()
    ok = np.flatnonzero(st == -1)
    say(t0, "instances passing the pivot test:", len(ok))
    assert len(ok) >= batch // 2
    gate = 1e-12 if precision == "fp64" else 1e-10
    worst = max(eta_inf(c, V[i], Xh[i, 0], B[i, 0]) for i in ok)
    say(t0, "worst eta over instances", worst)
    assert worst <= gate
    single = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, precision=prec)
    single.factorize(dev(c.values))
    for i in ok[[0, len(ok) // 2, -1]]:
        fb = s.factors(instance=int(i))
        rc, _ = single.refactorize(dev(V[i]))
        assert rc == 0
        fs = single.factors()
        assert np.array_equal(fb["Lx"], fs["Lx"]) and np.array_equal(fb["Ux"], fs["Ux"]), i
        if precision == "fp64":
            lu = oracle_refactor(oracle_mod, c, V[i], a0, EPS, a0["pivrow"])
            assert lu.nswaps == 0
            compare_factors(fb, lu)
    say(t0, "sampled instances equal their single refactorization")


@pytest.mark.timeout(1200)
def test_power_grid_1000_8rhs_full(ck, oracle_mod):
    t0 = time.time()
    c = mnagen.power_grid(1000, 1000, seed=0)
    nrhs = c.rhs.shape[0]
    say(t0, "power_grid_1000 n", c.n, "nnz", c.nnz, "nrhs", nrhs)
    assert nrhs == 8
    v = mnagen.restamp(c, 0, 4, 1)
    Bd = dev(c.rhs)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS)
    s.factorize(dev(c.values))
    a0 = s.analysis()
    say(t0, "fp64 factorized; dense tail", s.stats()["dense_tail"])
    rc, info = s.refactorize(dev(v))
    X = torch.zeros_like(Bd)
    s.solve(Bd, X, nrhs=nrhs)
    torch.cuda.synchronize()
    X64 = X.cpu().numpy()
    f = s.factors()
    piv = s.analysis()["pivrow"]
    s.close()
    say(t0, "fp64 refactorize rc", rc)
    lu = oracle_refactor(oracle_mod, c, v, a0, EPS, a0["pivrow"])
    say(t0, "oracle re-factorization done, swaps", lu.nswaps)
    assert lu.status == 0
    assert np.array_equal(piv, lu.pivrow)
    worst = compare_factors_sampled(f, lu)
    say(t0, "sampled scaled error", worst)
    kap = kappa_est(oracle_mod, lu, c, v, a0)
    xo = [oracle_mod.solve(lu, a0["rowperm_pre"], a0["colperm"], c.rhs[r]) for r in range(nrhs)]
    eo = [eta_inf(c, v, xo[r], c.rhs[r]) for r in range(nrhs)]
    for r in range(nrhs):
        e = eta_inf(c, v, X64[r], c.rhs[r])
        assert e <= 1e-12, (r, e)
        w = check_solution(X64[r], xo[r], kap, e, eo[r], "fp64 rhs %d" % r)
    say(t0, "fp64 solutions within the bound; kappa %.3e" % kap)
    s32 = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, precision=ck.CKTLU_FP32_IR, ir_tol=1e-10)
    s32.factorize(dev(c.values))
    rc, info = s32.refactorize(dev(v))
    X = torch.zeros_like(Bd)
    rc, sinfo = s32.solve(Bd, X, nrhs=nrhs)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    s32.close()
    etas = [eta_inf(c, v, Xh[r], c.rhs[r]) for r in range(nrhs)]
    say(t0, "fp32+ir rc", rc, "iters", sinfo.ir_iters, "fp64 fallback", sinfo.used_fp64, "eta", max(etas))
    assert max(etas) <= 1e-10
    ws = [check_solution(Xh[r], xo[r], kap, etas[r], eo[r], "fp32+ir rhs %d" % r) for r in range(nrhs)]
    say(t0, "fp32+ir forward difference / bound, worst %.3e" % max(ws))
