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
