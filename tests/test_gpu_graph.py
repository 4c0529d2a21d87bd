"""The captured batched NR step (cktlu_step_batched_graph) against the same
work issued eagerly: the graph is replayed several times with new values in
the same buffers, with eager work and synchronisations in between, and every
replay must equal the eager result (FP64: bit for bit; FP32 + refinement: each
instance within its eta gate, and equal to the eager refinement after as many
steps)."""
import numpy as np
import pytest

import mnagen

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


@pytest.mark.parametrize("tail", [-1, 100])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_graph_step_replays_match_eager(ck, oracle_mod, precision, tail):
    c = mnagen.mesh_transistor(30, 30, seed=16)
    batch, nrhs = 16, 2
    prec = ck.CKTLU_FP64 if precision == "fp64" else ck.CKTLU_FP32_IR
    g = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail, precision=prec, ir_tol=1e-10)
    e = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS, dense_tail=tail, precision=prec, ir_tol=1e-10)
    g.factorize(dev(c.values))
    e.factorize(dev(c.values))
    rng = np.random.default_rng(16)
    B = rng.standard_normal((batch, nrhs, c.n))
    Bd = dev(B)
    vals = torch.zeros((batch, c.nnz), dtype=torch.float64, device="cuda:0")      # the graph's buffers
    status = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
    X = torch.zeros((batch, nrhs, c.n), dtype=torch.float64, device="cuda:0")
    eta = torch.zeros(batch, dtype=torch.float64, device="cuda:0")
    for rep in range(3):
        V = mnagen.instance_values(c, batch, 0.2, seed=100 + rep)
        vals.copy_(dev(V))
        g.step_batched_graph(batch, vals, status, nrhs, Bd, X, eta, ir_steps=2)
        torch.cuda.synchronize()
        # eager work between the replays
        st_e = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
        X_e = torch.zeros_like(X)
        eta_e = torch.zeros(batch, dtype=torch.float64, device="cuda:0")
        e.refactorize_batched(batch, dev(V), st_e)
        e.solve_batched(batch, nrhs, Bd, X_e, st_e, eta_e)
        torch.cuda.synchronize()
        st, st_eh = status.cpu().numpy(), st_e.cpu().numpy()
        assert np.array_equal(st, st_eh)
        ok = np.flatnonzero(st == -1)
        assert len(ok) >= batch // 2
        Xh, Xe = X.cpu().numpy(), X_e.cpu().numpy()
        if precision == "fp64":
            assert np.array_equal(Xh[ok], Xe[ok]), rep
            assert np.all(eta.cpu().numpy() == -1.0)
        else:
            eh = eta.cpu().numpy()
            for i in ok:
                etas = [oracle_mod.backward_error(c.colptr, c.rowind, V[i], Xh[i, r], B[i, r]) for r in range(nrhs)]
                assert max(etas) <= 1e-10 and eh[i] <= 1e-10, (rep, i, etas, eh[i])
            # the eager refinement took the same steps (two at most here): same numbers
            assert np.allclose(Xh[ok], Xe[ok], rtol=1e-9, atol=0)
    g.close()
    e.close()


@pytest.mark.parametrize("batch", [1, 8])
def test_autotune_keeps_fastest_schedule_and_results(ck, oracle_mod, batch):
    """The autotuner measures several dense-block orders, keeps the fastest, and
    the factors and solutions with the tuned schedule still meet the gates."""
    c = mnagen.mesh_transistor(60, 60, seed=17)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=EPS)
    s.factorize(dev(c.values))
    V = mnagen.instance_values(c, batch, 0.2, seed=17)
    r = s.autotune(batch, dev(V if batch > 1 else V[0]), reps=2)
    assert len(r["dense_tail"]) >= 3 and len(set(r["dense_tail"])) == len(r["dense_tail"])
    assert r["ms_per_step"][r["best"]] == min(r["ms_per_step"])
    assert s.stats()["dense_tail"] == r["best_dense_tail"]
    # second stage: every knob left at its default was tried, and a kept value is one that was tried
    tried = {(k, v) for k, v, _ in r["knob_trials"]}
    for name in ("sweep_supernodes", "sweep_panel_rows", "solve_split_entries"):
        assert any(k == name for k, _ in tried), name
        kept = r["kept"][name]
        assert kept == 0 or (name, kept) in tried, (name, kept)
    status = torch.zeros(batch, dtype=torch.int32, device="cuda:0")
    s.refactorize_batched(batch, dev(V), status)
    B = np.repeat(c.rhs[:1][None], batch, axis=0)
    X = torch.zeros((batch, 1, c.n), dtype=torch.float64, device="cuda:0")
    s.solve_batched(batch, 1, dev(B), X, status)
    torch.cuda.synchronize()
    st, Xh = status.cpu().numpy(), X.cpu().numpy()
    for i in np.flatnonzero(st == -1):
        assert oracle_mod.backward_error(c.colptr, c.rowind, V[i], Xh[i, 0], B[i, 0]) <= 1e-12
