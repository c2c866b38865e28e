"""Algorithm 1 on the GPU (method FLR_METHOD_CHOLESKY): X^T X formed once on
the matrix cores, then per MM iteration the dense system Q = X^T X +
lambda1 A + lambda2 B factored by a blocked Cholesky and solved exactly.
Against the oracle's Algorithm 1 (dense Cholesky, section 3.1) at the FP64
parity bar: same status and MM count, max |d beta| <= 1e-8 ||beta||,
objective within 1e-11, or within twice the oracle's own rounding spread on
the case where that is larger (n < p leaves X^T X singular, and after many
MM iterations the weights make Q ill-conditioned enough that summation order
alone moves beta past 1e-8).  Sizes span several 64-wide blocks and ragged
tails (the factor's padding is the identity)."""
import numpy as np
import pytest

import flrgen
import oracle
from spread import oracle_with_spread

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def flr():
    import torch

    assert torch.cuda.is_available()
    import paper_1306_1970_amd as m

    return m


@pytest.fixture(scope="module")
def ctx(flr):
    c = flr.Context(0)
    yield c
    c.close()


def _check(flr, sol, ref, what):
    scale = np.max(np.abs(ref.beta))
    err = np.max(np.abs(sol.beta - ref.beta)) / scale
    ferr = abs(sol.objective - ref.objective) / ref.objective
    bar = max(1e-8, 2.0 * getattr(ref, "spread", 0.0))
    fbar = max(1e-11, 2.0 * getattr(ref, "fspread", 0.0))
    print("  %s gpu alg1 mm=%d f=%.15g | oracle alg1 mm=%d f=%.15g | err=%.2e (bar %.2e) f err=%.2e (bar %.2e)" % (
        what, sol.mm_iters, sol.objective, ref.mm_iters, ref.objective, err, bar, ferr, fbar), flush=True)
    want = {oracle.OK: flr.FLR_OK, oracle.MAX_ITER: flr.FLR_ERR_MAX_ITER}[ref.status]
    assert sol.status == want
    assert sol.mm_iters == ref.mm_iters
    assert sol.cg_iters == 0
    assert err <= bar
    assert ferr <= fbar


@pytest.mark.parametrize("graph,n,p,dtype,l1,l2", [
    ("chain", 80, 300, flrgen.F64, 0.2, 0.6),      # 5 blocks, ragged last block
    ("chain", 150, 257, flrgen.F32, 0.3, 0.8),     # one element past four blocks
    ("allpairs", 40, 60, flrgen.F64, 0.3, 0.05),   # the general edge set Algorithm 1 is meant for
    ("lattice", 300, 1024, flrgen.BF16, 0.2, 0.4),  # 16 blocks, bf16 X widened in the Gram product
])
def test_alg1_matches_oracle(flr, ctx, graph, n, p, dtype, l1, l2):
    inst = flrgen.small_instance(n, p, graph, dtype=dtype, seed=121, lam1=l1, lam2=l2)
    prob = flr.Problem.from_instance(ctx, inst)
    fp0 = prob.footprint
    sol = prob.solve(l1, l2, tol=1e-8, method=flr.FLR_METHOD_CHOLESKY)
    assert prob.footprint > fp0  # X^T X and the system are charged to the handle
    alg2 = prob.solve(l1, l2, tol=1e-8, inner_tol=1e-12)
    prob.close()
    ref = oracle_with_spread(inst, l1, l2, tol=1e-8, method=oracle.ALG1)
    _check(flr, sol, ref, "%s n=%d p=%d" % (graph, n, p))
    # Algorithm 2 with exact inner solves follows the same MM trajectory
    assert alg2.mm_iters == sol.mm_iters
    assert np.max(np.abs(alg2.beta - sol.beta)) <= 1e-7 * np.max(np.abs(sol.beta))


def test_alg1_flsa_and_warm_start(flr, ctx):
    # X = I (X^T X = I) with lambda1 = 0, where Algorithm 2's M is singular; then a warm start
    rng = np.random.default_rng(5)
    p = 200
    y = rng.uniform(-2, 2, 5)[np.minimum(np.arange(p) * 5 // p, 4)] + 0.3 * rng.standard_normal(p)
    e = flrgen.chain_edges(p)
    prob = flr.Problem.flsa(ctx, y, e)
    sol = prob.solve(0.0, 0.7, tol=1e-8, method=flr.FLR_METHOD_CHOLESKY)
    b0 = 0.5 * y
    warm = prob.solve(0.1, 0.7, tol=1e-8, method=flr.FLR_METHOD_CHOLESKY, warm_start=b0)
    prob.close()
    P = oracle.Problem(np.eye(p), oracle.F64, y, e)
    _check(flr, sol, oracle.solve(P, 0.0, 0.7, tol=1e-8, method=oracle.ALG1), "flsa lambda1=0")
    _check(flr, warm, oracle.solve(P, 0.1, 0.7, tol=1e-8, method=oracle.ALG1, beta0=b0), "flsa warm start")


def test_alg1_limits_and_unsupported_entry_points(flr, ctx):
    inst = flrgen.small_instance(4, 8193, "chain", dtype=flrgen.F32, seed=1)
    prob = flr.Problem.from_instance(ctx, inst)
    with pytest.raises(flr.FlrError) as ei:
        prob.solve(0.1, 0.1, tol=1e-6, method=flr.FLR_METHOD_CHOLESKY)
    assert ei.value.status == flr.FLR_ERR_INVALID_ARG
    prob.close()
    small = flrgen.small_instance(20, 50, "chain", dtype=flrgen.F64, seed=2)
    prob = flr.Problem.from_instance(ctx, small)
    with pytest.raises(flr.FlrError):
        prob.solve_grid(np.array([0.1]), np.array([0.2]), tol=1e-6, method=flr.FLR_METHOD_CHOLESKY)
    with pytest.raises(flr.FlrError):
        prob.solve(0.1, 0.2, tol=1e-6, method=7)
    prob.close()


def test_profile_dense(flr, ctx):
    inst = flrgen.small_instance(100, 500, "chain", dtype=flrgen.F64, seed=3)
    prob = flr.Problem.from_instance(ctx, inst)
    with pytest.raises(flr.FlrError):  # no Algorithm 1 workspace yet
        flr.flr_profile_dense(prob.h, 0.1, 0.5, 2)
    sol = prob.solve(0.1, 0.5, tol=1e-8, method=flr.FLR_METHOD_CHOLESKY)
    us = flr.flr_profile_dense(prob.h, 0.1, 0.5, 5)
    print("  p=500 assembly %.1f us, factor %.1f us, triangular solves %.1f us" % us, flush=True)
    assert all(t > 0.0 for t in us)
    # the iterate is untouched: a warm restart from it stops after one MM iteration, and MM descent from
    # the stored point lowers f by no more than the tolerance (beta itself may still drift along the
    # slowly converging fused directions, so it is not compared)
    again = prob.solve(0.1, 0.5, tol=1e-8, method=flr.FLR_METHOD_CHOLESKY, use_last=1)
    prob.close()
    assert again.mm_iters == 1
    assert again.objective <= sol.objective
    assert sol.objective - again.objective <= 1e-8 * sol.objective


def test_alg1_through_server_and_path(flr, ctx):
    # an all-pairs problem (the graph Algorithm 1 is meant for): one request through the serving loop with
    # method = Algorithm 1, then a three-point warm-started path, each against the oracle's Algorithm 1
    inst = flrgen.small_instance(50, 60, "allpairs", dtype=flrgen.F64, seed=131)
    prob = flr.Problem.from_instance(ctx, inst)
    P = oracle.Problem.from_instance(inst)
    srv = flr.flr_server_create(ctx.h, prob.footprint + (64 << 20), 2)
    o = flr.default_opts(method=flr.FLR_METHOD_CHOLESKY)
    t = flr.flr_server_submit(srv, prob.h, 0.3, 0.05, 1e-8, o)
    beta = np.zeros(inst.p)
    st, res = flr.flr_server_poll(srv, t, True, beta)
    flr.flr_server_destroy(srv)
    ref = oracle.solve(P, 0.3, 0.05, tol=1e-8, method=oracle.ALG1)

    class _S:
        pass

    s = _S()
    s.beta, s.status, s.objective, s.mm_iters, s.cg_iters = beta, st, res.objective, res.mm_iters, res.cg_iters
    _check(flr, s, ref, "server allpairs")
    l1 = np.array([0.5, 0.3, 0.1])
    l2 = np.array([0.02, 0.05, 0.1])
    st, betas, results = prob.solve_path(l1, l2, tol=1e-8, method=flr.FLR_METHOD_CHOLESKY)
    prob.close()
    b0 = None
    for k in range(l1.size):
        ref = oracle.solve(P, l1[k], l2[k], tol=1e-8, method=oracle.ALG1, beta0=b0)
        s = _S()
        r = results[k]
        s.beta, s.status, s.objective, s.mm_iters, s.cg_iters = betas[k], r["status"], r["objective"], r["mm_iters"], r["cg_iters"]
        _check(flr, s, ref, "path point %d" % k)
        b0 = ref.beta


def test_alg1_graph_replay_matches_eager(flr, ctx, monkeypatch):
    # every MM step of Algorithm 1 replays one captured graph; the eager launches (FLR_DENSE_GRAPH=0) must
    # give the same bits, and so must a second graph solve after the eager one on the same handle
    inst = flrgen.small_instance(90, 330, "allpairs", dtype=flrgen.F32, seed=141, lam1=0.3, lam2=0.02)
    prob = flr.Problem.from_instance(ctx, inst)
    g1 = prob.solve(0.3, 0.02, tol=1e-9, method=flr.FLR_METHOD_CHOLESKY)
    monkeypatch.setenv("FLR_DENSE_GRAPH", "0")
    e1 = prob.solve(0.3, 0.02, tol=1e-9, method=flr.FLR_METHOD_CHOLESKY)
    monkeypatch.delenv("FLR_DENSE_GRAPH")
    g2 = prob.solve(0.3, 0.02, tol=1e-9, method=flr.FLR_METHOD_CHOLESKY)
    prob.close()
    print("  graph mm=%d, eager mm=%d" % (g1.mm_iters, e1.mm_iters), flush=True)
    assert g1.mm_iters > 10
    for s in (g1, g2):
        assert (s.status, s.mm_iters, s.objective) == (e1.status, e1.mm_iters, e1.objective)
        assert np.array_equal(s.beta, e1.beta)
