"""The autotuner on the GPU: it times candidate launch shapes with the
library's own profiler, writes its cache, and a problem created from the
cached shapes still solves to the oracle's answer at the parity bar (the
shapes change only how X is tiled, never the method)."""
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


def test_tuned_shapes_keep_parity(flr, tmp_path, monkeypatch):
    from paper_1306_1970_amd import autotune

    monkeypatch.setenv("FLR_TUNE_CACHE", str(tmp_path / "tune.json"))
    inst = flrgen.small_instance(300, 3000, "chain", dtype=flrgen.F32, seed=55, lam1=0.3, lam2=0.7)
    ctx = flr.Context(0)
    entry = autotune.tune(ctx, inst.X, inst.dtype, inst.y, inst.edges, inst.lam1, inst.lam2, candidates=(64, 256, 1024),
                          reps=5, log=lambda m: print(m, flush=True))
    assert entry["target_wg_a"] in (64, 256, 1024) and entry["target_wg_b"] in (64, 256, 1024)
    assert autotune.lookup(inst.n, inst.p, inst.dtype) == entry
    ref = oracle.solve(oracle.Problem.from_instance(inst), inst.lam1, inst.lam2, tol=1e-8, inner_tol=1e-12,
                       method=oracle.ALG2)
    for cand in (64, 1024, None):  # two fixed shapes, then the cached tuned one (use_tuned)
        with autotune.launch_shape(cand, cand):
            prob = flr.Problem(ctx, inst.X, inst.dtype, inst.y, inst.edges, use_tuned=cand is None)
        sol = prob.solve(inst.lam1, inst.lam2, tol=1e-8, inner_tol=1e-12)
        prob.close()
        err = np.max(np.abs(sol.beta - ref.beta)) / np.max(np.abs(ref.beta))
        print("  shape %s: mm=%d (oracle %d) err=%.2e" % (cand, sol.mm_iters, ref.mm_iters, err), flush=True)
        assert sol.status == flr.FLR_OK and sol.mm_iters == ref.mm_iters
        assert err <= 1e-8
    ctx.close()
