"""The oracle's rounding spread on one case, used as the parity bar where a
problem is ill-conditioned enough that summation order alone moves beta
beyond the fixed FP64 bar.  The spread is the largest change of beta (and of
the objective) when the oracle runs with every product summed in reverse
order (columns of X and the graph renumbered p-1-j), or with y moved by one
ulp in random directions.  A GPU result is held to twice that, or to the
fixed bar where that is larger."""
import numpy as np

import oracle


def reversed_problem(inst):
    p = inst.p
    return oracle.Problem(np.ascontiguousarray(inst.X[:, ::-1]), inst.dtype, inst.y,
                          np.ascontiguousarray((p - 1 - inst.edges)[:, ::-1]))


def oracle_with_spread(inst, lam1, lam2, ulp_samples=2, **kw):
    """oracle.solve on inst, with .spread (beta, relative to max |beta|) and .fspread (objective, relative)."""
    ref = oracle.solve(oracle.Problem.from_instance(inst), lam1, lam2, **kw)
    runs = [(oracle.solve(reversed_problem(inst), lam1, lam2, **kw), True)]
    rng = np.random.default_rng(7)
    for _ in range(ulp_samples):
        y2 = inst.y + np.spacing(inst.y) * rng.choice([-1.0, 1.0], size=inst.n)
        runs.append((oracle.solve(oracle.Problem(inst.X, inst.dtype, y2, inst.edges), lam1, lam2, **kw), False))
    scale = max(np.max(np.abs(ref.beta)), 1e-300)
    ref.spread = 0.0
    ref.fspread = 0.0
    for r, rev in runs:
        assert r.mm_iters == ref.mm_iters
        ref.spread = max(ref.spread, float(np.max(np.abs((r.beta[::-1] if rev else r.beta) - ref.beta)) / scale))
        ref.fspread = max(ref.fspread, abs(r.objective - ref.objective) / abs(ref.objective))
    return ref
