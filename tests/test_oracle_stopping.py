"""Pins of the oracle's stopping rules against a closed-form MM trajectory.

With orthonormal columns (X^T X = I) and lambda2 = 0 the linear system of
section 3.1 is diagonal, so one MM step has the closed form

    beta_j <- z_j / (1 + lambda1 / (|beta_j| + eps)),   z = X^T y,

starting from the initialization beta_j = X_j^T y / X_j^T X_j = z_j, and the
FLR objective is f(b) = 1/2 (||y - X z||^2 + ||z - b||^2) + lambda1 ||b||_1.
That gives f at every iterate, the relative change of Algorithm 2's outer
test, and hence the iteration at which the outer test stops for any delta.

For each plausible misreading of the outer test (the perturbed objective in
place of f, the relative change taken over f_new instead of f_old, a bar ten
times too loose) the test picks a delta at which the misreading stops at a
different iteration than the stated rule, with a margin far above rounding,
and checks the oracle's MM count, iterate and objective there.  Both
algorithms are pinned.  A last test pins the repeat-until form of the inner
loop of Algorithm 2 on a one-coordinate problem, where a single PCG step is
an exact solve.
"""
import numpy as np
import pytest

import oracle

LAM = 0.3


def _orthonormal_problem(seed=4, n=12, p=6):
    rng = np.random.default_rng(seed)
    Xo, _ = np.linalg.qr(rng.standard_normal((n, p)))
    z_target = np.array([2.0, -0.05, 0.7, -1.3, 0.45, 0.0])[:p]
    y = Xo @ z_target + (np.eye(n) - Xo @ Xo.T) @ rng.standard_normal(n)
    return Xo, y


def _closed_form(Xo, y, lam, eps, iters):
    """Iterates, f and f_eps along the MM trajectory (orthonormal X, lambda2 = 0)."""
    z = Xo.T @ y
    resid2 = float(np.sum((y - Xo @ z) ** 2))
    b = z.copy()
    bs = [b]
    for _ in range(iters):
        b = z / (1.0 + lam / (np.abs(b) + eps))
        bs.append(b)
    quad = np.array([0.5 * (resid2 + np.sum((z - v) ** 2)) for v in bs])
    f = quad + lam * np.array([np.sum(np.abs(v)) for v in bs])
    fe = quad + lam * np.array([np.sum(np.abs(v) - eps * np.log1p(np.abs(v) / eps)) for v in bs])
    return bs, f, fe


def _rules(f, fe):
    d = np.abs(np.diff(f))
    return {
        "stated": d / f[:-1],                    # |f_new - f_old| / |f_old| <= delta
        "perturbed_f": np.abs(np.diff(fe)) / fe[:-1],
        "over_f_new": d / f[1:],
        "ten_times_looser": d / f[:-1] / 10.0,   # i.e. RE <= 10 delta
    }


def _stop(values, delta):
    """MM count at which a rule with these per-step values first passes delta (None: never)."""
    k = np.nonzero(values <= delta)[0]
    return int(k[0]) + 1 if k.size else None


def _discriminating_deltas(rules, mutant, lo=1e-9, margin=1.01, limit=4):
    """Deltas at which the stated rule and the mutant stop at different MM counts, each at least
    `margin` (relative) away from every per-step value of both rules."""
    vals = np.sort(np.concatenate([rules["stated"], rules[mutant]]))
    vals = vals[vals > lo]
    out = []
    for a, b in reversed(list(zip(vals[:-1], vals[1:]))):
        if b / a < margin * margin:
            continue
        delta = float(np.sqrt(a * b))
        s0, s1 = _stop(rules["stated"], delta), _stop(rules[mutant], delta)
        if s0 is not None and s0 != s1:
            out.append((delta, s0, s1))
        if len(out) >= limit:
            break
    return out


@pytest.mark.parametrize("mutant", ["perturbed_f", "over_f_new", "ten_times_looser"])
@pytest.mark.parametrize("method", [oracle.ALG1, oracle.ALG2])
def test_outer_stopping_rule_closed_form(mutant, method):
    eps = 1e-3  # large enough that f and f_eps change by visibly different amounts per step
    Xo, y = _orthonormal_problem()
    bs, f, fe = _closed_form(Xo, y, LAM, eps, 400)
    rules = _rules(f, fe)
    cases = _discriminating_deltas(rules, mutant)
    assert cases, "no delta separates the stated rule from " + mutant
    P = oracle.Problem(Xo, oracle.F64, y, np.zeros((0, 2), np.int64))
    for delta, s_stated, s_mut in cases:
        r = oracle.solve(P, LAM, 0.0, eps=eps, tol=delta, inner_tol=1e-15, method=method)
        scale = np.max(np.abs(bs[s_stated]))
        print("  %s delta=%.6g: stated rule stops at %d, %s at %s; oracle %d" % (
            mutant, delta, s_stated, mutant, s_mut, r.mm_iters))
        assert r.status == oracle.OK
        assert r.mm_iters == s_stated
        assert np.max(np.abs(r.beta - bs[s_stated])) <= 1e-12 * scale
        assert abs(r.objective - f[s_stated]) <= 1e-13 * f[s_stated]
        assert r.rel_change == pytest.approx(rules["stated"][s_stated - 1], rel=1e-9)


@pytest.mark.parametrize("eps", [1e-8, 1e-3])
def test_long_trajectory_count(eps):
    # a tight delta: many MM steps, the count still equals the closed form's
    Xo, y = _orthonormal_problem(seed=6)
    bs, f, fe = _closed_form(Xo, y, LAM, eps, 3000)
    rules = _rules(f, fe)
    delta = 1e-9
    want = _stop(rules["stated"], delta)
    assert want is not None and want > 10
    # keep clear of a near tie at the stopping step
    assert rules["stated"][want - 1] < delta / 1.01 and rules["stated"][want - 2] > delta * 1.01
    P = oracle.Problem(Xo, oracle.F64, y, np.zeros((0, 2), np.int64))
    for method in (oracle.ALG1, oracle.ALG2):
        r = oracle.solve(P, LAM, 0.0, eps=eps, tol=delta, inner_tol=1e-15, method=method)
        assert r.mm_iters == want
        assert np.max(np.abs(r.beta - bs[want])) <= 1e-11 * np.max(np.abs(bs[want]))


def test_inner_loop_is_repeat_until():
    # One coordinate, no edges: Q = x^T x + lambda1 / (|b| + eps) is a scalar and one PCG step solves
    # Q b = x^T y exactly (nu = M / Q, so x_1 = x_0 + r_0 / Q = c / Q).  A warm start next to the MM
    # fixed point already meets the inner tolerance; Algorithm 2's inner loop is repeat-until, so one
    # step still runs and the MM step returns the closed-form update c / Q(b0), not b0 itself.
    x = np.array([[0.8], [-1.1], [0.5]])
    y = np.array([1.3, -2.0, 0.4])
    s, c = float(x[:, 0] @ x[:, 0]), float(x[:, 0] @ y)
    lam, eps = 0.4, 1e-8
    b = c / s
    for _ in range(500):
        b = c / (s + lam / (abs(b) + eps))
    b0 = b * (1.0 + 1e-9)
    r0 = c - (s + lam / (abs(b0) + eps)) * b0
    assert 0.0 < abs(r0) / abs(c) < 1e-7
    want = c / (s + lam / (abs(b0) + eps))
    assert abs(want - b0) > 1e-10 * abs(b0)  # the one step moves the iterate
    P = oracle.Problem(x, oracle.F64, y, np.zeros((0, 2), np.int64))
    r = oracle.solve(P, lam, 0.0, eps=eps, tol=1e-3, inner_tol=1e-6, method=oracle.ALG2, beta0=np.array([b0]),
                     trajectory=True, max_iter=1)
    assert r.traj["cg"][0] == 1
    assert r.cg_iters == 1
    assert abs(r.beta[0] - want) <= 4e-16 * abs(want)
