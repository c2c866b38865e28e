"""Oracle parity on the code paths the full-size workloads take.

The small parity cases of test_gpu_parity.py do not reach every branch that
the benchmark configurations run: the headline chain at n = 1000, p = 10^4;
the 100 x 100 lattice, whose banded factor (bandwidth 100) uses every block
of the register-panel factorization's trailing triangle; more than 12 row-panel partial sums per
column panel and column panels of more than 256 rows in the X^T u kernel
(the c4 shape); requests through the serving loop; zero columns of X and
non-finite warm starts.  Where the oracle would need minutes for a whole
solve, both sides stop after the same capped number of MM iterations and the
iterates are compared there (status MAX_ITER on both sides).

Bar: same status and MM count; max |d beta| <= max(1e-8, 2 s) ||beta||,
where s is the oracle's own rounding spread on the same case - the largest
change of its beta when it runs with the columns of X (and the edge labels)
in reverse order, which sums every product in another order, or with y
moved by one ulp in random directions.  Early MM iterates (the first
few steps, where the weights 1/(|b| + eps) still move by orders of
magnitude) amplify rounding to about 1e-8 on some of these cases, in the
oracle as much as on the GPU.  Converged solves are also held to the
objective bar (1e-11 relative); a capped iterate is not stationary, so there
the reported objective must instead be f of the returned beta.
Inner tolerance 1e-12 on both sides.
"""
import numpy as np
import pytest

import flrgen
import oracle
from spread import oracle_with_spread as _oracle

pytestmark = pytest.mark.gpu

TOL_BETA = 1e-8
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


class _Sol:
    """A GPU result in one shape for _check."""

    def __init__(self, beta, status, objective, mm_iters, cg_iters):
        self.beta, self.status, self.objective, self.mm_iters, self.cg_iters = beta, status, objective, mm_iters, cg_iters


def _check(flr, sol, ref, inst, lam1, lam2, what=""):
    scale = max(np.max(np.abs(ref.beta)), 1e-300)
    err = np.max(np.abs(np.asarray(sol.beta) - ref.beta)) / scale
    bar = max(TOL_BETA, 2.0 * getattr(ref, "spread", 0.0))
    print("  %s gpu mm=%d cg=%d f=%.15g | oracle mm=%d cg=%d f=%.15g | err=%.3g (oracle spread %.2g, bar %.2g)" %
          (what, sol.mm_iters, sol.cg_iters, sol.objective, ref.mm_iters, ref.cg_iters, ref.objective, err,
           getattr(ref, "spread", float("nan")), bar), flush=True)
    want = {oracle.OK: flr.FLR_OK, oracle.MAX_ITER: flr.FLR_ERR_MAX_ITER}[ref.status]
    assert sol.status == want
    assert sol.mm_iters == ref.mm_iters
    assert err <= bar
    if ref.status == oracle.OK:
        assert abs(sol.objective - ref.objective) <= 1e-11 * abs(ref.objective)
    else:
        f_own = oracle.objective(oracle.Problem.from_instance(inst), lam1, lam2, np.asarray(sol.beta))
        assert abs(sol.objective - f_own) <= 1e-12 * abs(f_own)


def test_config2_full_size(flr, ctx):
    # the headline instance itself (seed 2, n = 1000, p = 10^4, AR(1) X stored FP32), first 3 MM iterations
    inst = flrgen.config2()
    print("case %s capped at 3 MM iterations" % inst.name, flush=True)
    prob = flr.Problem.from_instance(ctx, inst)
    sol = prob.solve(inst.lam1, inst.lam2, tol=inst.tol, inner_tol=INNER, max_iter=3)
    prob.close()
    # one spread sample here (each oracle run at this size takes tens of seconds)
    ref = _oracle(inst, inst.lam1, inst.lam2, ulp_samples=0, tol=inst.tol, inner_tol=INNER, max_iter=3,
                  method=oracle.ALG2)
    assert ref.status == oracle.MAX_ITER
    _check(flr, sol, ref, inst, inst.lam1, inst.lam2, "c2")


def _lattice100(seed=101, n=150):
    return flrgen.small_instance(n, 10000, "lattice", dtype=flrgen.F64, seed=seed, lam1=0.2, lam2=0.5, q=100)


def test_lattice_q100_banded(flr, ctx):
    # bandwidth 100 (W = 101): the band factor runs in register panels with its window in LDS
    inst = _lattice100()
    print("case %s capped at 4 MM iterations" % inst.name, flush=True)
    prob = flr.Problem.from_instance(ctx, inst)
    sol = prob.solve(inst.lam1, inst.lam2, tol=1e-10, inner_tol=INNER, max_iter=4)
    prob.close()
    ref = _oracle(inst, inst.lam1, inst.lam2, tol=1e-10, inner_tol=INNER, max_iter=4, method=oracle.ALG2)
    _check(flr, sol, ref, inst, inst.lam1, inst.lam2, "q=100")
    assert abs(sol.cg_iters - ref.cg_iters) <= max(5, ref.cg_iters // 50)


def test_lattice_q100_grid(flr, ctx):
    inst = _lattice100(seed=102)
    l1 = np.array([0.1, 0.3, 0.6, 1.0])
    l2 = np.array([0.5, 0.2, 0.8, 0.1])
    print("case %s grid B=4 capped at 3 MM iterations" % inst.name, flush=True)
    prob = flr.Problem.from_instance(ctx, inst)
    st, beta, res = prob.solve_grid(l1, l2, tol=1e-10, inner_tol=INNER, max_iter=3)
    prob.close()
    for b in range(l1.size):
        ref = _oracle(inst, l1[b], l2[b], tol=1e-10, inner_tol=INNER, max_iter=3, method=oracle.ALG2)
        r = res[b]
        _check(flr, _Sol(beta[b], r["status"], r["objective"], r["mm_iters"], r["cg_iters"]), ref, inst, l1[b], l2[b],
               "col %d" % b)


def test_lattice_wider_than_the_band_window(flr, ctx):
    # a 120 x 120 lattice: bandwidth 120 (W = 121) is wider than the register-panel factor's LDS window
    # (W <= 107), so M is factored by the blocked path (panels of 16 pivots in LDS, rank-16 updates in
    # global memory), single solve and grid
    inst = flrgen.small_instance(60, 14400, "lattice", dtype=flrgen.F32, seed=41, lam1=0.3, lam2=0.5)
    print("case %s W=121" % inst.name, flush=True)
    prob = flr.Problem.from_instance(ctx, inst)
    sol = prob.solve(0.3, 0.5, tol=1e-8, inner_tol=INNER, max_iter=6)
    l1 = np.array([0.3, 0.1, 1.0, 0.5])
    l2 = np.array([0.5, 0.2, 0.3, 2.0])
    st, beta, res = prob.solve_grid(l1, l2, tol=1e-8, inner_tol=INNER, max_iter=4)
    prob.close()
    ref = _oracle(inst, 0.3, 0.5, ulp_samples=1, tol=1e-8, inner_tol=INNER, max_iter=6, method=oracle.ALG2)
    _check(flr, sol, ref, inst, 0.3, 0.5, "single")
    for b in range(l1.size):
        ref = _oracle(inst, l1[b], l2[b], ulp_samples=0, tol=1e-8, inner_tol=INNER, max_iter=4, method=oracle.ALG2)
        r = res[b]
        _check(flr, _Sol(beta[b], r["status"], r["objective"], r["mm_iters"], r["cg_iters"]), ref, inst, l1[b], l2[b],
               "col %d" % b)


@pytest.mark.parametrize("dtype,n,p", [(flrgen.F64, 300, 7000), (flrgen.BF16, 120, 26000)])
def test_wide_panels_fp64(flr, ctx, dtype, n, p):
    # one row panel per column panel of X^T u (all n rows, > 256 for f64) and more than 12 partial
    # sums of X v per row (p_pad / (256 V) = 14 for f64, 13 for bf16): the branches the c4 shape takes
    from paper_1306_1970_amd import autotune

    inst = flrgen.small_instance(n, p, "chain", dtype=dtype, seed=81, lam1=0.5, lam2=1.0)
    print("case %s one X^T u row panel" % inst.name, flush=True)
    with autotune.launch_shape(target_b=1):
        prob = flr.Problem(ctx, inst.X, inst.dtype, inst.y, inst.edges, use_tuned=False)
    sol = prob.solve(inst.lam1, inst.lam2, tol=1e-10, inner_tol=INNER, max_iter=6)
    prob.close()
    ref = _oracle(inst, inst.lam1, inst.lam2, tol=1e-10, inner_tol=INNER, max_iter=6, method=oracle.ALG2)
    _check(flr, sol, ref, inst, inst.lam1, inst.lam2, "panels")


def test_wide_panels_mixed(flr, ctx):
    # the same branches with FP32 inner products: the objective gap to the FP64 oracle stays <= 1e-6
    from paper_1306_1970_amd import autotune

    inst = flrgen.small_instance(300, 7000, "chain", dtype=flrgen.F64, seed=82, lam1=0.5, lam2=1.0)
    with autotune.launch_shape(target_b=1):
        prob = flr.Problem(ctx, inst.X, inst.dtype, inst.y, inst.edges, use_tuned=False)
    sol = prob.solve(inst.lam1, inst.lam2, tol=1e-6, precision=flr.FLR_PREC_MIXED_FP32)
    prob.close()
    P = oracle.Problem.from_instance(inst)
    ref = oracle.solve(P, inst.lam1, inst.lam2, tol=1e-6, method=oracle.ALG2)
    gap = (oracle.objective(P, inst.lam1, inst.lam2, sol.beta) - ref.objective) / ref.objective
    print("  mixed mm=%d cg=%d gap=%.2e | oracle mm=%d cg=%d" % (sol.mm_iters, sol.cg_iters, gap, ref.mm_iters,
                                                                   ref.cg_iters), flush=True)
    assert sol.status == flr.FLR_OK
    assert abs(gap) <= 1e-6


def test_serving_requests_match_oracle(flr, ctx):
    # one request per graph type through the continuous-batching server, each against the oracle
    insts = [
        (flrgen.serving_cell(1000, "chain", seed=91, scale=0.3), 0.2, 0.4),
        (flrgen.serving_cell(1000, "lattice", seed=92, scale=0.2), 0.1, 0.3),
        (flrgen.small_instance(30, 40, "allpairs", dtype=flrgen.F64, seed=7), 0.3, 0.05),
    ]
    probs = [flr.Problem.from_instance(ctx, i) for i, _, _ in insts]
    srv = flr.flr_server_create(ctx.h, sum(p.footprint for p in probs), 3)
    o = flr.default_opts(inner_tol=INNER)
    tickets = [flr.flr_server_submit(srv, p.h, a, b, 1e-7, o) for p, (_, a, b) in zip(probs, insts)]
    for t, p, (inst, a, b) in zip(tickets, probs, insts):
        beta = np.zeros(p.p)
        st, res = flr.flr_server_poll(srv, t, True, beta)
        ref = oracle.solve(oracle.Problem.from_instance(inst), a, b, tol=1e-7, inner_tol=INNER)
        _check(flr, _Sol(beta, st, res.objective, res.mm_iters, res.cg_iters), ref, inst, a, b, inst.name)
    flr.flr_server_destroy(srv)
    for p in probs:
        p.close()


def test_zero_columns(flr, ctx):
    # zero columns of X: the initialization gives beta_j = 0 there, the penalties alone decide them
    inst = flrgen.small_instance(80, 300, "chain", dtype=flrgen.F64, seed=93, lam1=0.2, lam2=0.6)
    inst.X[:, 7] = 0.0
    inst.X[:, 150] = 0.0
    inst.y = inst.X @ inst.beta_true + np.random.default_rng(1).standard_normal(inst.n)
    prob = flr.Problem.from_instance(ctx, inst)
    sol = prob.solve(inst.lam1, inst.lam2, tol=1e-8, inner_tol=INNER)
    prob.close()
    ref = oracle.solve(oracle.Problem.from_instance(inst), inst.lam1, inst.lam2, tol=1e-8, inner_tol=INNER,
                       method=oracle.ALG2)
    _check(flr, sol, ref, inst, inst.lam1, inst.lam2, "zero columns")


@pytest.mark.parametrize("where", ["host", "device"])
def test_nan_warm_start_is_a_numerical_failure(flr, ctx, where):
    import torch

    inst = flrgen.small_instance(40, 200, "chain", dtype=flrgen.F64, seed=94)
    b0 = np.zeros(inst.p)
    b0[17] = np.nan
    ws = b0 if where == "host" else torch.from_numpy(b0).to("cuda:0")
    prob = flr.Problem.from_instance(ctx, inst)
    sol = prob.solve(inst.lam1, inst.lam2, tol=1e-8, warm_start=ws)
    assert sol.status == flr.FLR_ERR_NUMERICAL
    # the handle stays usable
    ok = prob.solve(inst.lam1, inst.lam2, tol=1e-6)
    assert ok.status == flr.FLR_OK
    # the grid reports it per column
    st, beta, res = prob.solve_grid(np.array([0.1, 0.2]), np.array([0.3, 0.3]), tol=1e-6,
                                    warm_start=np.stack([b0, np.zeros(inst.p)]))
    assert res[0]["status"] == flr.FLR_ERR_NUMERICAL and res[1]["status"] == flr.FLR_OK
    prob.close()
