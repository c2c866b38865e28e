#!/usr/bin/env python3
"""Writes grid_oracle_spread.json: the FP64 oracle's own rounding spread on
the grid parity instances (Algorithm 2, tol 1e-7, inner 1e-12).

For every (lambda1, lambda2) column the oracle is run three more times on the
same mathematical problem with different rounding: once with the columns of X
(and the edge labels) in reverse order, which changes the summation order of
every product, and twice with y moved by one ulp in random directions.  The
spread is the largest relative beta change and objective change among them.
Where the MM trajectory is rounding-sensitive (weights 1/(|b|+eps) near
zero), any implementation differs from the oracle by about this much.  Calls
only the oracle and the seeded input generator.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import flrgen  # noqa: E402
import oracle  # noqa: E402

INSTANCES = [(80, 600, flrgen.F64), (120, 2500, flrgen.F32), (60, 4100, flrgen.BF16)]
VALS = [0.05, 0.4, 1.5]


def reversed_problem(inst):
    p = inst.p
    X = np.ascontiguousarray(inst.X[:, ::-1])
    E = np.ascontiguousarray((p - 1 - inst.edges)[:, ::-1])
    return oracle.Problem(X, inst.dtype, inst.y, E)


def main():
    out = {"what": "oracle rounding spread per grid column (Algorithm 2, tol 1e-7, inner 1e-12, "
                   "max_cg 20p): max over reversed summation order and two one-ulp moves of y",
           "instances": []}
    for n, p, dt in INSTANCES:
        inst = flrgen.small_instance(n, p, "chain", dtype=dt, seed=31)
        l1, l2 = flrgen.grid_lambdas(np.array(VALS))
        P = oracle.Problem.from_instance(inst)
        R = reversed_problem(inst)
        rng = np.random.default_rng(0)
        cols = []
        for b in range(l1.size):
            kw = dict(tol=1e-7, inner_tol=1e-12, method=oracle.ALG2, max_cg=20 * p)
            ref = oracle.solve(P, l1[b], l2[b], **kw)
            sc = float(np.max(np.abs(ref.beta)))
            runs = [(oracle.solve(R, l1[b], l2[b], **kw), True)]
            for _ in range(2):
                y2 = inst.y + np.spacing(inst.y) * rng.choice([-1.0, 1.0], size=inst.n)
                runs.append((oracle.solve(oracle.Problem(inst.X, inst.dtype, y2, inst.edges), l1[b], l2[b], **kw),
                             False))
            db, dobj, mms = 0.0, 0.0, []
            for r, rev in runs:
                beta = r.beta[::-1] if rev else r.beta
                db = max(db, float(np.max(np.abs(beta - ref.beta))) / sc)
                dobj = max(dobj, abs(r.objective - ref.objective) / ref.objective)
                mms.append(int(r.mm_iters))
            cols.append({"lambda1": float(l1[b]), "lambda2": float(l2[b]), "mm_iters": int(ref.mm_iters),
                         "beta_spread": db, "objective_spread": dobj, "perturbed_mm_iters": mms})
            print("n=%d p=%d col %d: mm %d beta spread %.2e objective spread %.2e" % (
                n, p, b, ref.mm_iters, db, dobj), flush=True)
        out["instances"].append({"n": n, "p": p, "dtype": dt, "seed": 31, "columns": cols})
    with open(os.path.join(HERE, "grid_oracle_spread.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
