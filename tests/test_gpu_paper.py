"""The paper's simulation scenarios on the GPU (section 5.1: C1-C3 on a chain,
p = 200; section 5.2: C4 on a 16 x 16 lattice; n = 1000, relative objective
change 1e-5, eps 1e-8).  At the paper's own setting (inner tolerance equal to
the outer one) the GPU's MM count must equal the oracle's on every data set
and setting; with exact inner solves (1e-12) beta and f must also meet the
FP64 parity bar, or twice the oracle's own rounding spread where that is
larger.  The comparison of these counts with the paper's printed means is the
oracle's (tests/test_oracle_paper_counts.py); the larger sizes are measured
by bench.py --workload paper."""
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


SMALL = [("C1", 200), ("C2", 200), ("C3", 200), ("C4", 16)]


@pytest.mark.parametrize("scenario,size", SMALL)
def test_counts_at_the_papers_setting(flr, ctx, scenario, size):
    mism = []
    for d in range(10):
        inst = flrgen.paper_scenario(scenario, size, d)
        prob = flr.Problem.from_instance(ctx, inst)
        P = oracle.Problem.from_instance(inst)
        for lp in flrgen.PAPER_LAMBDAS:
            g = prob.solve(lp[0], lp[1], tol=flrgen.PAPER_TOL, eps=1e-8)
            o = oracle.solve(P, lp[0], lp[1], eps=1e-8, tol=flrgen.PAPER_TOL, method=oracle.ALG2)
            assert g.status == flr.FLR_OK and o.status == oracle.OK
            if g.mm_iters != o.mm_iters:
                mism.append((d, lp, g.mm_iters, o.mm_iters))
            assert abs(g.objective - o.objective) <= 1e-6 * o.objective
        prob.close()
    print("  %s size %d: 40 solves, MM count differences %s" % (scenario, size, mism), flush=True)
    assert not mism


@pytest.mark.parametrize("scenario,size", SMALL)
def test_parity_with_exact_inner_solves(flr, ctx, scenario, size):
    inst = flrgen.paper_scenario(scenario, size, 0)
    prob = flr.Problem.from_instance(ctx, inst)
    for lp in flrgen.PAPER_LAMBDAS:
        g = prob.solve(lp[0], lp[1], tol=flrgen.PAPER_TOL, eps=1e-8, inner_tol=1e-12)
        ref = oracle_with_spread(inst, lp[0], lp[1], ulp_samples=6, eps=1e-8, tol=flrgen.PAPER_TOL, inner_tol=1e-12,
                                 method=oracle.ALG2)
        scale = np.max(np.abs(ref.beta))
        err = np.max(np.abs(g.beta - ref.beta)) / scale
        bar = max(1e-8, 2 * ref.spread)
        fbar = max(1e-11, 2 * ref.fspread)
        print("  %s lam=%s mm %d/%d err %.2e (bar %.2e) f err %.2e" % (
            scenario, lp, g.mm_iters, ref.mm_iters, err, bar, abs(g.objective - ref.objective) / ref.objective))
        assert g.status == flr.FLR_OK and g.mm_iters == ref.mm_iters
        assert err <= bar
        assert abs(g.objective - ref.objective) <= fbar * ref.objective
    prob.close()
