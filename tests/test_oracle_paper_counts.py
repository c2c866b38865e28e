"""The oracle against the iteration counts the paper prints (Appendix C,
Tables C.1-C.3, MM column): scenarios C1-C3 of section 5.1 at n = 1000,
p = 200, ten data sets per scenario, the four (lambda1, lambda2) settings,
relative objective change 1e-5 and eps 1e-8 (section 5), inner tolerance
equal to the outer one, Algorithm 2.  The data sets are new draws from the
scenario's generating equation, not the paper's, so the comparison is of
means: every cell within 0.75 iterations of the printed mean and no overall
bias.  At p = 200 the printed means are 3.0 to 4.4, so a count that is off by
one, a stopping rule taken on another quantity or weights that move the MM
trajectory fail here.  C4 (the lattice) is not pinned: at q = 16 the printed
counts are 2 to 4 iterations above this start's (they fit a start from zero),
while at q = 32 they agree; that reading is recorded with the measurements."""
import json
import os

import numpy as np
import pytest

import flrgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables_c.json")


def _printed(scenario, size):
    cells = json.load(open(GOLDEN))["cells"]
    return {(c["lambda1"], c["lambda2"]): c for c in cells if c["scenario"] == scenario and c["size"] == size}


def test_fixture_is_the_four_tables():
    d = json.load(open(GOLDEN))
    assert "Tables C.1-C.4" in d["source"]
    assert len(d["cells"]) == 3 * 16 + 16
    c = _printed("C1", 200)[(0.1, 0.1)]
    assert (c["mm_iters"], c["mmgpu_iters"], c["mmgpu_seconds"]) == (3.0, 3.0, 0.2858)
    assert _printed("C4", 128)[(1.0, 1.0)]["mm_iters"] == 109.0


@pytest.mark.parametrize("scenario", ["C1", "C2", "C3"])
def test_mm_counts_match_tables(scenario):
    printed = _printed(scenario, 200)
    diffs = []
    for lp in flrgen.PAPER_LAMBDAS:
        counts = []
        for d in range(10):
            inst = flrgen.paper_scenario(scenario, 200, d)
            r = oracle.solve(oracle.Problem.from_instance(inst), lp[0], lp[1], eps=1e-8, tol=flrgen.PAPER_TOL,
                             method=oracle.ALG2)
            assert r.status == oracle.OK
            counts.append(r.mm_iters)
        mean = float(np.mean(counts))
        want = printed[lp]["mm_iters"]
        print("  %s p=200 lam=%s mean MM %.2f (%s) | printed %.1f" % (scenario, lp, mean, counts, want))
        assert abs(mean - want) <= 0.75
        diffs.append(mean - want)
    assert abs(np.mean(diffs)) <= 0.35
