"""Serving loop: requests submitted while others run are admitted as slots
and HBM budget free up, their work overlaps on the device, and every result is
the same alone and in the mix (cold starts; each problem has its own buffers
and fixed reduction trees, so the results are bitwise equal)."""
import threading
import time

import numpy as np
import pytest

import flrgen
import oracle

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


def _problems(flr, ctx):
    insts = [
        flrgen.serving_cell(1000, "chain", seed=51, scale=0.3),
        flrgen.serving_cell(1000, "lattice", seed=52, scale=0.2),
        flrgen.serving_cell(1000, "allpairs", seed=53, scale=0.05),
        flrgen.serving_cell(5000, "chain", seed=54, scale=0.2),
    ]
    return insts, [flr.Problem.from_instance(ctx, i) for i in insts]


def test_alone_equals_mix(flr, ctx):
    insts, probs = _problems(flr, ctx)
    rng = np.random.default_rng(5)
    reqs = [(k, float(10 ** rng.uniform(-1.5, 0.5)), float(10 ** rng.uniform(-1.5, 0.5))) for k in range(len(probs))
            for _ in range(3)]
    tol = 1e-6
    opts = dict(max_cg=20000)
    alone = []
    for k, l1, l2 in reqs:
        s = probs[k].solve(l1, l2, tol=tol, **opts)
        alone.append(s)
    budget = sum(p.footprint for p in probs)
    srv = flr.flr_server_create(ctx.h, budget, 4)
    o = flr.default_opts(**opts)
    tickets = []
    for k, l1, l2 in reqs:
        tickets.append(flr.flr_server_submit(srv, probs[k].h, l1, l2, tol, o))
    outs = []
    for t, (k, l1, l2) in zip(tickets, reqs):
        beta = np.zeros(probs[k].p)
        st, res = flr.flr_server_poll(srv, t, True, beta)
        outs.append((st, res, beta))
    flr.flr_server_destroy(srv)
    for (st, res, beta), a, (k, l1, l2) in zip(outs, alone, reqs):
        print("  %-22s lam=(%.3g,%.3g) alone mm=%d mix mm=%d" % (insts[k].name, l1, l2, a.mm_iters, res.mm_iters),
              flush=True)
        assert st == a.status
        assert res.mm_iters == a.mm_iters and res.cg_iters == a.cg_iters
        assert np.array_equal(beta, a.beta)
        assert res.objective == a.objective
    for p in probs:
        p.close()


def test_admission_respects_budget(flr, ctx):
    insts, probs = _problems(flr, ctx)
    fps = [p.footprint for p in probs]
    budget = max(fps) + min(fps)  # at most two small or one large problem at a time
    srv = flr.flr_server_create(ctx.h, budget, 4)
    o = flr.default_opts(max_cg=20000)
    tickets = [flr.flr_server_submit(srv, probs[k].h, 0.3, 0.3, 1e-5, o) for k in range(len(probs)) for _ in range(2)]
    peak = [0]
    stop = [False]

    def watch():
        while not stop[0]:
            q, r, b = flr.flr_server_stats(srv)
            peak[0] = max(peak[0], b)
            time.sleep(0.0005)

    th = threading.Thread(target=watch)
    th.start()
    for t in tickets:
        st, res = flr.flr_server_poll(srv, t, True)
        assert st == flr.FLR_OK
    stop[0] = True
    th.join()
    q, r, b = flr.flr_server_stats(srv)
    flr.flr_server_destroy(srv)
    print("  budget %d peak in use %d" % (budget, peak[0]), flush=True)
    assert peak[0] <= budget
    assert q == 0 and r == 0 and b == 0
    for p in probs:
        p.close()


def test_oversized_request_is_rejected(flr, ctx):
    insts, probs = _problems(flr, ctx)
    srv = flr.flr_server_create(ctx.h, 1 << 20, 2)
    with pytest.raises(flr.FlrError) as ei:
        flr.flr_server_submit(srv, probs[3].h, 0.1, 0.1, 1e-6)
    assert ei.value.status == flr.FLR_ERR_BUSY
    flr.flr_server_destroy(srv)
    for p in probs:
        p.close()


def test_poll_not_ready_and_unknown_ticket(flr, ctx):
    insts, probs = _problems(flr, ctx)
    srv = flr.flr_server_create(ctx.h, 1 << 34, 1)
    o = flr.default_opts(max_cg=20000)
    t1 = flr.flr_server_submit(srv, probs[3].h, 0.05, 0.05, 1e-8, o)
    t2 = flr.flr_server_submit(srv, probs[0].h, 0.05, 0.05, 1e-8, o)
    st, _ = flr.flr_server_poll(srv, t2, False)
    assert st in (flr.FLR_ERR_NOT_READY, flr.FLR_OK)
    assert flr.flr_server_poll(srv, t1, True)[0] == flr.FLR_OK
    assert flr.flr_server_poll(srv, t2, True)[0] == flr.FLR_OK
    with pytest.raises(flr.FlrError):
        flr.flr_server_poll(srv, 999999, False)
    flr.flr_server_destroy(srv)
    for p in probs:
        p.close()


def test_ragged_batch_equals_solo_solves(flr, ctx):
    # problems of uneven p and different graphs in one call: each result is the solo solve's
    insts = [
        flrgen.small_instance(120, 2000, "chain", dtype=flrgen.F32, seed=61, lam1=0.3, lam2=0.6),
        flrgen.small_instance(80, 400, "lattice", dtype=flrgen.F64, seed=62, lam1=0.2, lam2=0.4, q=20),
        flrgen.small_instance(40, 60, "allpairs", dtype=flrgen.F64, seed=63, lam1=0.5, lam2=0.05),
        flrgen.small_instance(60, 300, "chain", dtype=flrgen.BF16, seed=64, lam1=0.1, lam2=0.2),
    ]
    l1 = [i.lam1 for i in insts]
    l2 = [i.lam2 for i in insts]
    solo = []
    for inst, a, b in zip(insts, l1, l2):
        p = flr.Problem.from_instance(ctx, inst)
        solo.append(p.solve(a, b, tol=1e-7))
        p.close()
    probs = [flr.Problem.from_instance(ctx, i) for i in insts]
    betas = [np.zeros(i.p) for i in insts]
    st, res = flr.flr_solve_batch(probs, l1, l2, 1e-7, betas=betas)
    for k, (s1, r, bta) in enumerate(zip(solo, res, betas)):
        print("  %-28s solo mm=%d cg=%d | batch mm=%d cg=%d" % (insts[k].name, s1.mm_iters, s1.cg_iters, r.mm_iters,
                                                                 r.cg_iters), flush=True)
        assert r.status == s1.status
        assert r.mm_iters == s1.mm_iters and r.cg_iters == s1.cg_iters
        assert np.array_equal(bta, s1.beta)
        assert r.objective == s1.objective
    # the same batch with exact inner solves against the oracle (Algorithm 2, FP64 bar)
    o = flr.default_opts(inner_tol=1e-12)
    betas = [np.zeros(i.p) for i in insts]
    st, res = flr.flr_solve_batch(probs, l1, l2, 1e-7, opts=o, betas=betas)
    for inst, a, b, r, bta in zip(insts, l1, l2, res, betas):
        ref = oracle.solve(oracle.Problem.from_instance(inst), a, b, tol=1e-7, inner_tol=1e-12, method=oracle.ALG2)
        err = np.max(np.abs(bta - ref.beta)) / np.max(np.abs(ref.beta))
        print("  %-28s batch mm=%d | oracle mm=%d err=%.2e" % (inst.name, r.mm_iters, ref.mm_iters, err), flush=True)
        assert r.status == flr.FLR_OK and r.mm_iters == ref.mm_iters
        assert err <= 1e-8
        assert abs(r.objective - ref.objective) <= 1e-11 * ref.objective
    with pytest.raises(flr.FlrError) as ei:  # the same handle twice
        flr.flr_solve_batch([probs[0], probs[0]], [0.1, 0.2], [0.1, 0.2], 1e-6)
    assert ei.value.status == flr.FLR_ERR_INVALID_ARG
    for p in probs:
        p.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_ragged_batch_in_grouped_launches(flr, ctx, precision):
    # 18 problems over all three stored types, chain / lattice (banded M) / all pairs, p from 40 to 3000:
    # one graph of grouped launches drives them all, and every result must equal its solo solve bit for bit
    rng = np.random.default_rng(71)
    insts, lam = [], []
    specs = [("chain", 150, 3000), ("chain", 60, 300), ("lattice", 80, 400), ("allpairs", 30, 40), ("chain", 200, 1200),
             ("lattice", 60, 144)]
    for k in range(18):
        graph, n, p = specs[k % len(specs)]
        dtype = (flrgen.F64, flrgen.F32, flrgen.BF16)[k % 3]
        inst = flrgen.small_instance(n, p, graph, dtype=dtype, seed=700 + k)
        insts.append(inst)
        lam.append((float(rng.uniform(0.05, 0.6)), float(rng.uniform(0.05, 0.8))))
    prec = flr.FLR_PREC_FP64 if precision == "fp64" else flr.FLR_PREC_MIXED_FP32
    o = flr.default_opts(precision=prec)
    probs = [flr.Problem.from_instance(ctx, i) for i in insts]
    solo = [p.solve(a, b, tol=1e-7, precision=prec) for p, (a, b) in zip(probs, lam)]
    betas = [np.zeros(i.p) for i in insts]
    st, res = flr.flr_solve_batch(probs, [a for a, _ in lam], [b for _, b in lam], 1e-7, opts=o, betas=betas)
    for p in probs:
        p.close()
    print("  %s: MM %s" % (precision, [r.mm_iters for r in res]), flush=True)
    for s1, r, bta in zip(solo, res, betas):
        assert r.status == s1.status == flr.FLR_OK
        assert (r.mm_iters, r.cg_iters, r.objective) == (s1.mm_iters, s1.cg_iters, s1.objective)
        assert np.array_equal(bta, s1.beta)


def test_grouped_batch_with_signal_approximation(flr, ctx):
    # X = I problems (no X stored; the grouped A launch only forms the direction) in one f64 group with an
    # explicit-X problem, chain and lattice graphs: every result equals its solo solve bit for bit
    rng = np.random.default_rng(17)
    y1 = rng.standard_normal(300)
    y2 = rng.standard_normal(400)
    dense = flrgen.small_instance(60, 500, "chain", dtype=flrgen.F64, seed=171)
    probs = [flr.Problem.flsa(ctx, y1, flrgen.chain_edges(300)), flr.Problem.flsa(ctx, y2, flrgen.lattice_edges(20)),
             flr.Problem.from_instance(ctx, dense)]
    lam = [(0.2, 0.5), (0.1, 0.3), (0.3, 0.6)]
    solo = [p.solve(a, b, tol=1e-8) for p, (a, b) in zip(probs, lam)]
    betas = [np.zeros(p.p) for p in probs]
    st, res = flr.flr_solve_batch(probs, [a for a, _ in lam], [b for _, b in lam], 1e-8, betas=betas)
    for p in probs:
        p.close()
    print("  MM %s" % [r.mm_iters for r in res], flush=True)
    for s1, r, bta in zip(solo, res, betas):
        assert r.status == s1.status == flr.FLR_OK
        assert (r.mm_iters, r.cg_iters, r.objective) == (s1.mm_iters, s1.cg_iters, s1.objective)
        assert np.array_equal(bta, s1.beta)
