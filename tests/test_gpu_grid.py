"""Batched (lambda1, lambda2) grid solves: every column against the FP64
oracle (same bar as the single-solve parity tests) and against the single
solve of the same column."""
import json
import os

import numpy as np
import pytest

import flrgen
import oracle

pytestmark = pytest.mark.gpu
INNER = 1e-12


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


def _grid(flr, ctx, inst, l1, l2, tol, **kw):
    prob = flr.Problem.from_instance(ctx, inst)
    st, beta, res = prob.solve_grid(l1, l2, tol=tol, **kw)
    singles = [prob.solve(a, b, tol=tol, **kw) for a, b in zip(l1, l2)]
    prob.close()
    return st, beta, res, singles


# Bars per column from the oracle's own rounding spread (tests/golden/grid_oracle_spread.json, written by
# make_grid_spread.py from the oracle alone): the oracle run with the columns of X in reverse order (every
# product summed in another order) and with y moved by one ulp.  Where the MM trajectory is insensitive the
# spread is below 1e-10 and the bar is the FP64 parity bar (beta 1e-8, objective 1e-11); on the few columns
# whose trajectory amplifies rounding (lambda1 = 0.05: weights 1/(|b| + eps) on coordinates near zero) no
# implementation can do better than that spread, and the bar is twice it.
with open(os.path.join(os.path.dirname(__file__), "golden", "grid_oracle_spread.json")) as _fh:
    SPREAD = json.load(_fh)


def _bars(n, p, dtype):
    for inst in SPREAD["instances"]:
        if (inst["n"], inst["p"], inst["dtype"]) == (n, p, dtype):
            return [(max(1e-8, 2.0 * c["beta_spread"]), max(1e-11, 2.0 * c["objective_spread"]))
                    for c in inst["columns"]]
    raise KeyError((n, p, dtype))


@pytest.mark.parametrize("n,p,dtype", [(80, 600, flrgen.F64), (120, 2500, flrgen.F32), (60, 4100, flrgen.BF16)])
def test_grid_chain_matches_oracle(flr, ctx, n, p, dtype):
    inst = flrgen.small_instance(n, p, "chain", dtype=dtype, seed=31)
    vals = np.array([0.05, 0.4, 1.5])
    l1, l2 = flrgen.grid_lambdas(vals)
    bars = _bars(n, p, dtype)
    print("grid %s B=%d" % (inst.name, l1.size), flush=True)
    # inner cap raised so that every inner solve really reaches 1e-12 (a capped, inexact
    # inner solve makes the MM trajectory depend on rounding detail)
    st, beta, res, singles = _grid(flr, ctx, inst, l1, l2, 1e-7, inner_tol=INNER, max_cg=20 * inst.p)
    P = oracle.Problem.from_instance(inst)
    for b in range(l1.size):
        ref = oracle.solve(P, l1[b], l2[b], tol=1e-7, inner_tol=INNER, method=oracle.ALG2, max_cg=20 * inst.p)
        err = np.max(np.abs(beta[b] - ref.beta)) / np.max(np.abs(ref.beta))
        err_single = np.max(np.abs(beta[b] - singles[b].beta)) / np.max(np.abs(singles[b].beta))
        ebar, obar = bars[b]
        print("  col %d lam=(%g,%g) grid mm=%d cg=%d | oracle mm=%d | single mm=%d | err=%.2e (bar %.1e) "
              "vs single %.2e" % (b, l1[b], l2[b], res[b]["mm_iters"], res[b]["cg_iters"], ref.mm_iters,
                                  singles[b].mm_iters, err, ebar, err_single), flush=True)
        assert res[b]["status"] == flr.FLR_OK
        assert res[b]["mm_iters"] == ref.mm_iters
        assert abs(res[b]["objective"] - ref.objective) <= obar * ref.objective
        assert err <= ebar
        # the single solve is another rounding of the same trajectory: within the bar of each, so twice
        assert err_single <= 2 * ebar


def test_grid_mixed_graphs_and_lambda1_zero(flr, ctx):
    # lattice graph and a lambda1 = 0 column (Jacobi) in one grid
    inst = flrgen.small_instance(60, 100, "lattice", dtype=flrgen.F64, seed=32)
    l1 = np.array([0.0, 0.2, 1.0])
    l2 = np.array([0.5, 0.3, 0.1])
    st, beta, res, singles = _grid(flr, ctx, inst, l1, l2, 1e-7, inner_tol=INNER, max_cg=100 * inst.p)
    P = oracle.Problem.from_instance(inst)
    for b in range(l1.size):
        ref = oracle.solve(P, l1[b], l2[b], tol=1e-7, inner_tol=INNER)
        err = np.max(np.abs(beta[b] - ref.beta)) / np.max(np.abs(ref.beta))
        print("  col %d grid mm=%d | oracle mm=%d err=%.2e" % (b, res[b]["mm_iters"], ref.mm_iters, err), flush=True)
        assert res[b]["mm_iters"] == ref.mm_iters
        assert err <= 1e-8


def test_grid_columns_finish_independently(flr, ctx):
    # very different lambdas converge after very different MM counts; a capped column reports MAX_ITER
    inst = flrgen.small_instance(50, 300, "chain", dtype=flrgen.F64, seed=33)
    l1 = np.array([0.01, 5.0, 0.3])
    l2 = np.array([0.01, 5.0, 0.3])
    prob = flr.Problem.from_instance(ctx, inst)
    # exact inner solves: with inner solves stopped at 1e-8 the capped iterates differ at ~1e-8
    # with the summation order of the products, which this test does not pin
    st, beta, res = prob.solve_grid(l1, l2, tol=1e-8, max_iter=40, inner_tol=INNER)
    single = [prob.solve(a, b, tol=1e-8, max_iter=40, inner_tol=INNER) for a, b in zip(l1, l2)]
    prob.close()
    for b in range(3):
        assert res[b]["status"] == single[b].status
        assert res[b]["mm_iters"] == single[b].mm_iters
        np.testing.assert_allclose(beta[b], single[b].beta, rtol=0, atol=1e-8 * np.max(np.abs(single[b].beta)) + 1e-300)


def test_grid_compaction_keeps_every_column(flr, ctx):
    # 48 columns with spread-out MM counts: finished columns are dropped from the
    # batched products several times during the solve; every column must still
    # equal its own single solve, and the result must not depend on the batch
    inst = flrgen.small_instance(40, 200, "chain", dtype=flrgen.F64, seed=34)
    vals = np.logspace(-2.0, 0.8, 7)
    l1, l2 = flrgen.grid_lambdas(vals)
    l1, l2 = l1[:48], l2[:48]
    prob = flr.Problem.from_instance(ctx, inst)
    st, beta, res = prob.solve_grid(l1, l2, tol=1e-9, inner_tol=INNER)
    st2, beta2, res2 = prob.solve_grid(l1[::-1].copy(), l2[::-1].copy(), tol=1e-9, inner_tol=INNER)
    mms = [r["mm_iters"] for r in res]
    print("  mm range %d..%d" % (min(mms), max(mms)), flush=True)
    assert max(mms) > 2 * min(mms)
    for b in range(l1.size):
        s1 = prob.solve(l1[b], l2[b], tol=1e-9, inner_tol=INNER)
        assert res[b]["status"] == s1.status == flr.FLR_OK
        assert res[b]["mm_iters"] == s1.mm_iters
        assert np.max(np.abs(beta[b] - s1.beta)) <= 1e-8 * np.max(np.abs(s1.beta))
        # the same column in the reversed batch: identical arithmetic per column
        rb = l1.size - 1 - b
        assert res2[rb]["mm_iters"] == res[b]["mm_iters"]
        assert np.array_equal(beta2[rb], beta[b])
    prob.close()


def test_grid_tiny_caps_report_max_iter(flr, ctx):
    # caps far below what the solve needs: the batch stops and every column reports MAX_ITER
    inst = flrgen.small_instance(40, 300, "lattice", dtype=flrgen.F32, seed=35)
    l1 = np.array([0.1, 1.0])
    l2 = np.array([0.2, 2.0])
    prob = flr.Problem.from_instance(ctx, inst)
    st, beta, res = prob.solve_grid(l1, l2, tol=1e-12, max_iter=1, max_cg=2)
    prob.close()
    assert st == flr.FLR_ERR_MAX_ITER
    for r in res:
        assert r["status"] == flr.FLR_ERR_MAX_ITER and r["mm_iters"] == 1 and r["cg_iters"] <= 2
    assert np.all(np.isfinite(beta))


def test_grid_lattice_banded(flr, ctx):
    # lattice columns apply M^-1 through the banded factor (one per column), default inner cap
    inst = flrgen.small_instance(80, 144, "lattice", dtype=flrgen.F32, seed=36)
    l1, l2 = flrgen.grid_lambdas(np.array([0.1, 0.6]))
    prob = flr.Problem.from_instance(ctx, inst)
    st, beta, res = prob.solve_grid(l1, l2, tol=1e-7, inner_tol=INNER)
    prob.close()
    P = oracle.Problem.from_instance(inst)
    for b in range(l1.size):
        ref = oracle.solve(P, l1[b], l2[b], tol=1e-7, inner_tol=INNER, method=oracle.ALG2)
        err = np.max(np.abs(beta[b] - ref.beta)) / np.max(np.abs(ref.beta))
        print("  col %d grid mm=%d cg=%d | oracle mm=%d cg=%d err=%.2e" % (
            b, res[b]["mm_iters"], res[b]["cg_iters"], ref.mm_iters, ref.cg_iters, err), flush=True)
        assert res[b]["status"] == flr.FLR_OK
        assert res[b]["mm_iters"] == ref.mm_iters
        assert err <= 1e-8
        assert abs(res[b]["cg_iters"] - ref.cg_iters) <= max(5, ref.cg_iters // 50)


def test_grid_lattice_held_boundaries(flr, ctx, monkeypatch):
    # nine banded columns: while at least eight run, a column that reaches its MM boundary waits for the
    # next shared boundary launch (every 16th); the held schedule must give every column the oracle's
    # solution and the unheld schedule's
    inst = flrgen.small_instance(80, 144, "lattice", dtype=flrgen.F32, seed=36)
    l1, l2 = flrgen.grid_lambdas(np.array([0.1, 0.6, 2.0]))
    prob = flr.Problem.from_instance(ctx, inst)
    st, beta, res = prob.solve_grid(l1, l2, tol=1e-7, inner_tol=INNER)
    monkeypatch.setenv("FLR_GRID_HOLD", "1")
    st1, beta1, res1 = prob.solve_grid(l1, l2, tol=1e-7, inner_tol=INNER)
    prob.close()
    assert st == flr.FLR_OK and st1 == flr.FLR_OK
    P = oracle.Problem.from_instance(inst)
    for b in range(l1.size):
        ref = oracle.solve(P, l1[b], l2[b], tol=1e-7, inner_tol=INNER, method=oracle.ALG2)
        scale = np.max(np.abs(ref.beta))
        err = np.max(np.abs(beta[b] - ref.beta)) / scale
        err1 = np.max(np.abs(beta[b] - beta1[b])) / scale
        print("  col %d held mm=%d cg=%d | unheld mm=%d cg=%d | oracle mm=%d err=%.2e vs unheld %.2e" % (
            b, res[b]["mm_iters"], res[b]["cg_iters"], res1[b]["mm_iters"], res1[b]["cg_iters"], ref.mm_iters,
            err, err1), flush=True)
        assert res[b]["mm_iters"] == ref.mm_iters == res1[b]["mm_iters"]
        # the products may come from different GEMM kernels (the number of active columns differs
        # between the schedules), so the two agree to rounding, not bit for bit
        assert abs(res[b]["cg_iters"] - res1[b]["cg_iters"]) <= 2
        assert err <= 1e-8 and err1 <= 1e-10


@pytest.mark.parametrize("graph,vals", [("chain", np.logspace(-2.0, 0.8, 7)), ("lattice", np.array([0.1, 0.6, 2.0]))])
def test_grid_graph_replay_matches_eager(flr, ctx, monkeypatch, graph, vals):
    # The allocating grid replays each polling period (8 batched steps) as a HIP graph, one per hold
    # pattern, captured again after every compaction.  The same solve with eager launches
    # (FLR_GRID_GRAPH=0) must give the same bits, and so must a second graph solve on the same handle
    # after eager work in between: every replay is checked against eager arithmetic.
    inst = flrgen.small_instance(40 if graph == "chain" else 80, 200 if graph == "chain" else 144, graph,
                                 dtype=flrgen.F64, seed=34 if graph == "chain" else 36)
    l1, l2 = flrgen.grid_lambdas(vals)
    l1, l2 = l1[:48], l2[:48]
    prob = flr.Problem.from_instance(ctx, inst)
    st_g, beta_g, res_g = prob.solve_grid(l1, l2, tol=1e-9, inner_tol=INNER)
    monkeypatch.setenv("FLR_GRID_GRAPH", "0")
    st_e, beta_e, res_e = prob.solve_grid(l1, l2, tol=1e-9, inner_tol=INNER)
    single = prob.solve(l1[0], l2[0], tol=1e-9, inner_tol=INNER)  # other eager work on the handle
    monkeypatch.delenv("FLR_GRID_GRAPH")
    st_g2, beta_g2, res_g2 = prob.solve_grid(l1, l2, tol=1e-9, inner_tol=INNER)
    prob.close()
    mms = [r["mm_iters"] for r in res_g]
    print("  %s: %d columns, MM %d..%d, PCG steps up to %d" % (graph, l1.size, min(mms), max(mms),
                                                              max(r["cg_iters"] for r in res_g)), flush=True)
    assert st_g == st_e == st_g2 == flr.FLR_OK
    assert np.array_equal(beta_g, beta_e) and np.array_equal(beta_g2, beta_e)
    for a, b, c in zip(res_g, res_e, res_g2):
        assert (a["mm_iters"], a["cg_iters"], a["objective"]) == (b["mm_iters"], b["cg_iters"], b["objective"])
        assert (c["mm_iters"], c["cg_iters"], c["objective"]) == (b["mm_iters"], b["cg_iters"], b["objective"])
    assert single.mm_iters == res_e[0]["mm_iters"]


def test_grid_workspace_is_charged_to_footprint(flr, ctx):
    # serving admission charges flr_problem_footprint: the grid workspace a handle keeps after a
    # grid solve (per-column vectors, products, band factors) must be part of it
    inst = flrgen.small_instance(40, 144, "lattice", dtype=flrgen.F32, seed=37)
    prob = flr.Problem.from_instance(ctx, inst)
    before = prob.footprint
    l1, l2 = np.array([0.1, 0.5, 1.0, 2.0]), np.array([0.2, 0.2, 0.3, 0.4])
    prob.solve_grid(l1, l2, tol=1e-5)
    after = prob.footprint
    print("  footprint %d -> %d bytes" % (before, after), flush=True)
    # at least the four columns' banded factors (by columns and by rows) and eight p-vectors each
    W = inst.meta["q"] + 1
    assert after - before >= 4 * (2 * inst.p * W + 8 * inst.p) * 8
    prob.close()


def test_grid_workspace_failure_leaves_the_handle_usable(flr, ctx):
    # A 509 x 509 lattice (bandwidth 510) with 256 columns asks for about 541 GB of per-column band
    # factors: the single workspace allocation fails with FLR_ERR_OUT_OF_MEMORY before any kernel runs.
    # The partial workspace must be released, so a small grid on the same handle then works.
    q = 509
    inst = flrgen.small_instance(2, q * q, "lattice", dtype=flrgen.F32, seed=38, q=q)
    prob = flr.Problem.from_instance(ctx, inst)
    fp0 = prob.footprint
    l1 = np.full(256, 0.5)
    l2 = np.full(256, 0.5)
    with pytest.raises(flr.FlrError) as ei:
        prob.solve_grid(l1, l2, tol=1e-4, max_iter=1, max_cg=2)
    assert ei.value.status == flr.FLR_ERR_OUT_OF_MEMORY
    assert prob.footprint == fp0
    st, beta, res = prob.solve_grid(l1[:2], l2[:2], tol=1e-4, max_iter=1, max_cg=2)
    prob.close()
    assert all(r["status"] in (flr.FLR_OK, flr.FLR_ERR_MAX_ITER) for r in res)
    assert np.all(np.isfinite(beta))
