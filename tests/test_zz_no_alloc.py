"""The allocation-free solve: cktlu_solve_noalloc through the C ABI gives the same
solutions as cktlu_solve (the same kernels, its work rows in the library's
file-scope device array instead of a buffer it allocates), on two calls in a row,
the second with a smaller circuit, and refuses what it cannot do without
allocating (no device factors yet, FP32 factors, more rows than the array holds)."""
import sys

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


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda:0")


def _ctx(ck, c, precision=0, tail=0):
    o = ck.cktlu_default_options()
    o.precision = precision
    o.dense_tail_size = tail
    ctx = ck.cktlu_create(o)
    assert ck.cktlu_analyze(ctx, c.n, c.colptr, c.rowind) == 0
    return ctx


@pytest.mark.parametrize("tail", [-1, 200])
def test_solve_noalloc_equals_solve(ck, oracle_mod, tail):
    cases = [mnagen.mesh_transistor(60, 60, seed=51), mnagen.mesh_vsrc(20, 20, 4, seed=52)]
    assert cases[1].n < cases[0].n                      # the second call: a smaller input
    for i, c in enumerate(cases):
        print("case", i, "n", c.n, "tail", tail, flush=True)
        sys.stdout.flush()
        ctx = _ctx(ck, c, tail=tail)
        try:
            v = dev(mnagen.restamp(c, 51 + i, 0, 1))
            assert ck.cktlu_factorize(ctx, dev(c.values)) == 0
            assert ck.cktlu_refactorize(ctx, v, None) == 0
            for nrhs in (1, 3, 8, 11):
                rng = np.random.default_rng(nrhs)
                B = dev(rng.standard_normal((nrhs, c.n)))
                X1 = torch.full((nrhs, c.n), 5.0, dtype=torch.float64, device="cuda:0")
                X2 = torch.full((nrhs, c.n), -5.0, dtype=torch.float64, device="cuda:0")
                assert ck.cktlu_solve(ctx, nrhs, B, c.n, X1, c.n, None) == 0
                assert ck.cktlu_solve_noalloc(ctx, nrhs, B, c.n, X2, c.n) == 0
                torch.cuda.synchronize()
                assert torch.equal(X1, X2), (i, nrhs)
                vh = v.cpu().numpy()
                Bh, Xh = B.cpu().numpy(), X2.cpu().numpy()
                for r in range(nrhs):
                    assert oracle_mod.backward_error(c.colptr, c.rowind, vh, Xh[r], Bh[r]) <= 1e-12
        finally:
            ck.cktlu_destroy(ctx)


def test_solve_noalloc_refusals(ck):
    c = mnagen.mesh_transistor(20, 20, seed=53)
    b = dev(c.rhs[0])
    x = torch.zeros(c.n, dtype=torch.float64, device="cuda:0")
    # factors only on the host: uploading them would allocate
    ctx = _ctx(ck, c)
    try:
        assert ck.cktlu_factorize_host(ctx, c.values) == 0
        assert ck.cktlu_solve_noalloc(ctx, 1, b, c.n, x, c.n) == ck.CKTLU_E_STATE
    finally:
        ck.cktlu_destroy(ctx)
    # FP32 factors need refinement vectors
    ctx = _ctx(ck, c, precision=ck.CKTLU_FP32_IR)
    try:
        assert ck.cktlu_factorize(ctx, dev(c.values)) == 0
        assert ck.cktlu_solve_noalloc(ctx, 1, b, c.n, x, c.n) == ck.CKTLU_E_STATE
    finally:
        ck.cktlu_destroy(ctx)
    # more rows than the file-scope array holds: a diagonal matrix of 2^19 + 1 rows
    n = (1 << 19) + 1
    cp = np.arange(n + 1, dtype=np.int32)
    ri = np.arange(n, dtype=np.int32)
    o = ck.cktlu_default_options()
    ctx = ck.cktlu_create(o)
    try:
        assert ck.cktlu_analyze(ctx, n, cp, ri) == 0
        assert ck.cktlu_factorize(ctx, dev(np.full(n, 2.0))) == 0
        bb = dev(np.ones(n))
        xx = torch.zeros(n, dtype=torch.float64, device="cuda:0")
        assert ck.cktlu_solve_noalloc(ctx, 1, bb, n, xx, n) == ck.CKTLU_E_LIMIT
        assert ck.cktlu_solve(ctx, 1, bb, n, xx, n, None) == 0
        torch.cuda.synchronize()
        assert float(xx.max()) == 0.5 and float(xx.min()) == 0.5
    finally:
        ck.cktlu_destroy(ctx)
