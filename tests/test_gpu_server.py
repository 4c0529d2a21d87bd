"""The request loop: several circuits of different sizes served together give
exactly the results each gives alone, with an HBM budget that forces requests
to wait for admission (never more resident than the budget allows)."""
import numpy as np
import pytest

import mnagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ck():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_14082_amd as m
    return m


def make_requests(nsteps=4):
    reqs = []
    for tag, (kind, n) in enumerate([(0, 900), (1, 2000), (2, 1600), (0, 3000), (2, 2500), (1, 1200)]):
        c = mnagen.mix_circuit(kind, n, seed=tag)
        vals = np.stack([mnagen.restamp(c, tag, 5, t) for t in range(nsteps)])
        reqs.append((tag, c, vals))
    return reqs


def run(ck, reqs, slots, budget, precision, nsteps=4):
    srv = ck.Server(slots=slots, hbm_budget_bytes=budget, precision=precision)
    out = {}
    bufs = []
    for tag, c, vals in reqs:
        v = torch.tensor(vals, device="cuda:0")
        b = torch.tensor(c.rhs[0], device="cuda:0")
        x = torch.zeros((nsteps, c.n), dtype=torch.float64, device="cuda:0")
        bufs.append((tag, x))
        srv.submit(tag, c.n, c.colptr, c.rowind, nsteps, v, b, x)
    done = []
    while len(done) < len(reqs):
        done += srv.poll(wait_ms=200)
    srv.close()
    torch.cuda.synchronize()
    for tag, x in bufs:
        out[tag] = x.cpu().numpy()
    return out, {d["tag"]: d for d in done}


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_mix_equals_alone_and_respects_budget(ck, oracle_mod, precision):
    prec = ck.CKTLU_FP64 if precision == "fp64" else ck.CKTLU_FP32_IR
    reqs = make_requests()
    alone, fps = {}, {}
    for r in reqs:
        x, d = run(ck, [r], slots=1, budget=0.0, precision=prec)
        assert d[r[0]]["status"] >= 0
        alone.update(x)
        fps[r[0]] = d[r[0]]["footprint"]
    # a budget that the largest request shares only with small ones and that the
    # whole set exceeds: admission has to wait for memory
    budget = 1.5 * max(fps.values())
    assert sum(fps.values()) > budget
    mixed, done = run(ck, reqs, slots=4, budget=budget, precision=prec)
    for tag, c, vals in reqs:
        assert done[tag]["status"] >= 0, done[tag]
        assert np.array_equal(mixed[tag], alone[tag]), tag
        gate = 1e-12 if precision == "fp64" else 1e-10
        for t in range(vals.shape[0]):
            assert oracle_mod.backward_error(c.colptr, c.rowind, vals[t], mixed[tag][t], c.rhs[0]) <= gate
    # resident footprints never exceed the budget (a request alone may)
    events = sorted([(d["admit_s"], 1, d["footprint"]) for d in done.values()] +
                    [(d["end_s"], 0, -d["footprint"]) for d in done.values()])
    used = 0
    for t, kind, f in events:
        used += f
        if kind == 1:
            assert used <= budget or used == f, (used, budget)
    # some requests overlapped on the device
    spans = [(d["admit_s"], d["end_s"]) for d in done.values()]
    assert any(a2 < e1 and a1 < e2 for i, (a1, e1) in enumerate(spans) for (a2, e2) in spans[i + 1:])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_served_solutions_vs_oracle(ck, oracle_mod, precision):
    """Solutions served in a mix with a circuit of n >= 100k equal the oracle's
    solutions of the same steps' matrices within the condition-scaled bound, and the
    large request's results are bitwise those it gives alone."""
    import sys
    import time
    from helpers import check_solution, kappa_est, oracle_refactor
    t0 = time.time()
    prec = ck.CKTLU_FP64 if precision == "fp64" else ck.CKTLU_FP32_IR
    nsteps = 3
    reqs = []
    for tag, (kind, n) in enumerate([(1, 120_000), (0, 2000), (2, 5000)]):
        c = mnagen.mix_circuit(kind, n, seed=40 + tag)
        vals = np.stack([mnagen.restamp(c, 40 + tag, 5, t) for t in range(nsteps)])
        reqs.append((tag, c, vals))
    print("sizes", [r[1].n for r in reqs], flush=True)
    assert reqs[0][1].n >= 100_000
    mixed, done = run(ck, reqs, slots=3, budget=0.0, precision=prec, nsteps=nsteps)
    alone, _ = run(ck, reqs[:1], slots=1, budget=0.0, precision=prec, nsteps=nsteps)
    assert np.array_equal(alone[0], mixed[0])
    print("[%5.1fs] served" % (time.time() - t0), flush=True)
    gate = 1e-12 if precision == "fp64" else 1e-10
    for tag, c, vals in reqs:
        assert done[tag]["status"] >= 0, done[tag]
        s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=1e-3)
        an = s.analysis(with_pivots=False)
        s.close()
        lu = oracle_mod.gp_lu(c.n, c.colptr, c.rowind, vals[0], an["rowperm_pre"], an["colperm"], 1e-3)
        for t in range(nsteps):
            lu = oracle_refactor(oracle_mod, c, vals[t], an, 1e-3, lu.pivrow)
            assert lu.status == 0
            b = c.rhs[0]
            x = mixed[tag][t]
            e = oracle_mod.backward_error(c.colptr, c.rowind, vals[t], x, b)
            assert e <= gate, (tag, t, e)
            xo = oracle_mod.solve(lu, an["rowperm_pre"], an["colperm"], b)
            eo = oracle_mod.backward_error(c.colptr, c.rowind, vals[t], xo, b)
            w = check_solution(x, xo, kappa_est(oracle_mod, lu, c, vals[t], an), e, eo, "req %d step %d" % (tag, t))
        print("[%5.1fs] request %d (n %d) within the bound, last ratio %.2e" % (time.time() - t0, tag, c.n, w),
              flush=True)
        sys.stdout.flush()
