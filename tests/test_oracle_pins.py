"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these re-types the oracle's formulas: each checks it against a
closed form, a hand-computed value, a theorem of the paper, brute force on
tiny inputs, or finite differences.  A dropped term, a wrong sign or index,
or a transposed operand in the oracle fails at least one of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import flrgen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
EPS = 1e-8


def _problem(X, y, edges, dtype=oracle.F64):
    return oracle.Problem(np.asarray(X, dtype=np.float64) if dtype == oracle.F64 else X, dtype, y,
                          np.asarray(edges, dtype=np.int64).reshape(-1, 2))


# --------------------------------------------------------------------------
# FLR objective: hand-computed example (golden fixture)
# --------------------------------------------------------------------------
def test_objective_hand_example():
    g = json.load(open(os.path.join(GOLD, "objective_tiny.json")))
    P = _problem(g["X"], g["y"], g["edges"])
    b = np.array(g["beta"])
    assert oracle.objective(P, g["lambda1"], g["lambda2"], b) == pytest.approx(g["f"], rel=1e-15)
    assert oracle.objective(P, g["lambda1"], 0.0, b) == pytest.approx(g["f_lambda2_zero"], rel=1e-15)
    # edge orientation must not matter (E is a set of unordered pairs)
    P2 = _problem(g["X"], g["y"], [[1, 0], [2, 1]])
    assert oracle.objective(P2, g["lambda1"], g["lambda2"], b) == pytest.approx(g["f"], rel=1e-15)


def test_objective_storage_types_are_exact():
    # f32 / bf16 storage is widened exactly: the same values stored three ways give one objective
    rng = np.random.default_rng(0)
    x64 = rng.standard_normal((7, 9))
    xb = flrgen.f64_to_bf16_bits(x64)
    xw = flrgen.bf16_bits_to_f64(xb)
    y = rng.standard_normal(7)
    b = rng.standard_normal(9)
    e = flrgen.chain_edges(9)
    f64 = oracle.objective(_problem(xw, y, e), 0.3, 0.7, b)
    f32 = oracle.objective(oracle.Problem(xw.astype(np.float32), oracle.F32, y, e), 0.3, 0.7, b)
    fbf = oracle.objective(oracle.Problem(xb, oracle.BF16, y, e), 0.3, 0.7, b)
    assert f64 == f32 == fbf


def test_perturbed_objective_limits():
    # |t| - eps log(1+|t|/eps) -> |t| as eps -> 0 (Proposition 1 (ii)); and it is 0 at t = 0
    g = json.load(open(os.path.join(GOLD, "objective_tiny.json")))
    P = _problem(g["X"], g["y"], g["edges"])
    b = np.array(g["beta"])
    f = oracle.objective(P, g["lambda1"], g["lambda2"], b)
    for eps in (1e-2, 1e-4, 1e-8):
        fe = oracle.objective_eps(P, g["lambda1"], g["lambda2"], eps, b)
        # each of the p + m terms loses at most eps*log(1+|t|/eps) <= eps*(1+log(1+4/eps))
        bound = (g["lambda1"] * 3 + g["lambda2"] * 2) * eps * (1 + math.log1p(4.0 / eps))
        assert 0.0 <= f - fe <= bound
    z = np.zeros(3)
    assert oracle.objective_eps(P, 1.0, 1.0, 1e-8, z) == pytest.approx(0.5 * np.sum(np.array(g["y"]) ** 2))


# --------------------------------------------------------------------------
# Proposition 1 (iii): the majorizer touches f_eps at the reference point and lies above it
# --------------------------------------------------------------------------
@pytest.mark.parametrize("graph", ["chain", "lattice", "allpairs"])
def test_majorization(graph):
    inst = flrgen.small_instance(12, 9 if graph == "lattice" else 8, graph, seed=3)
    P = oracle.Problem.from_instance(inst)
    rng = np.random.default_rng(1)
    for trial in range(20):
        ref = rng.standard_normal(inst.p) * rng.choice([1e-9, 1e-3, 1.0])
        if trial % 3 == 0:
            ref[::2] = 0.0  # exact zeros and ties
        b = rng.standard_normal(inst.p)
        fe_ref = oracle.objective_eps(P, 0.4, 0.9, EPS, ref)
        g_ref = oracle.surrogate(P, 0.4, 0.9, EPS, ref, ref)
        assert g_ref == pytest.approx(fe_ref, rel=1e-14, abs=1e-14)
        g = oracle.surrogate(P, 0.4, 0.9, EPS, b, ref)
        fe = oracle.objective_eps(P, 0.4, 0.9, EPS, b)
        assert g >= fe - 1e-12 * abs(fe)


# --------------------------------------------------------------------------
# The linear system (linear-system equation) is the stationarity condition of the majorizer:
# grad g_eps(b | ref) = Q(ref) b - c, checked by central differences of the majorizer (exact for a quadratic)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("graph", ["chain", "lattice", "allpairs"])
def test_system_is_majorizer_gradient(graph):
    inst = flrgen.small_instance(10, 9 if graph == "lattice" else 7, graph, seed=5)
    P = oracle.Problem.from_instance(inst)
    rng = np.random.default_rng(2)
    ref = rng.standard_normal(inst.p)
    ref[1] = ref[2]  # a fused pair
    Q, c = oracle.system(P, 0.3, 0.6, 1e-2, ref)  # eps large so the curvature is moderate
    assert np.allclose(Q, Q.T)
    assert np.all(np.linalg.eigvalsh(Q) > 0)
    b = rng.standard_normal(inst.p)
    h = 1e-3
    fd = np.zeros(inst.p)
    for j in range(inst.p):
        e = np.zeros(inst.p)
        e[j] = h
        fd[j] = (oracle.surrogate(P, 0.3, 0.6, 1e-2, b + e, ref) - oracle.surrogate(P, 0.3, 0.6, 1e-2, b - e, ref)) / (2 * h)
    np.testing.assert_allclose(Q @ b - c, fd, rtol=1e-7, atol=1e-7)


def test_gradient_eps_matches_finite_differences():
    inst = flrgen.small_instance(9, 7, "chain", seed=8)
    P = oracle.Problem.from_instance(inst)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(inst.p)
    eps = 1e-2
    g = oracle.gradient_eps(P, 0.5, 0.8, eps, b)
    h = 1e-5
    for j in range(inst.p):
        e = np.zeros(inst.p)
        e[j] = h
        fd = (oracle.objective_eps(P, 0.5, 0.8, eps, b + e) - oracle.objective_eps(P, 0.5, 0.8, eps, b - e)) / (2 * h)
        assert g[j] == pytest.approx(fd, rel=1e-6, abs=1e-6)


def test_initialization_ratio():
    # X with orthogonal columns of norms s_j: beta0_j = X_j^T y / s_j^2 (initialization of Algorithms 1 and 2)
    s = np.array([1.0, 2.0, 0.5, 3.0])
    X = np.zeros((6, 4))
    for j in range(4):
        X[j, j] = s[j]
    X[5, :] = 0.0
    y = np.array([1.0, -2.0, 3.0, 0.25, 7.0, 9.0])
    P = _problem(X, y, [])
    np.testing.assert_allclose(oracle.init_beta(P), y[:4] / s, rtol=1e-15)
    # a zero column gives 0
    X[:, 2] = 0.0
    b0 = oracle.init_beta(_problem(X, y, []))
    assert b0[2] == 0.0


# --------------------------------------------------------------------------
# lambda2 = 0 with orthonormal X: per-coordinate closed form of the f_eps minimizer (Hunter-Li MM, section 3.1)
# --------------------------------------------------------------------------
def _eps_soft(z, lam, eps):
    t = abs(z) - lam - eps
    disc = math.sqrt(t * t + 4.0 * abs(z) * eps)
    mag = (t + disc) / 2.0 if t >= 0 else 2.0 * abs(z) * eps / (disc - t)
    return math.copysign(mag, z)


@pytest.mark.parametrize("method", [oracle.ALG1, oracle.ALG2])
def test_lasso_orthonormal_closed_form(method):
    rng = np.random.default_rng(4)
    n, p = 12, 6
    Xo, _ = np.linalg.qr(rng.standard_normal((n, p)))
    z_target = np.array([2.0, -0.05, 0.7, -1.3, 0.45, 0.0])
    y = Xo @ z_target + (np.eye(n) - Xo @ Xo.T) @ rng.standard_normal(n)
    P = _problem(Xo, y, [])
    lam = 0.3
    r = oracle.solve(P, lam, 0.0, tol=0.0, max_iter=3000, inner_tol=1e-14, method=method)
    z = Xo.T @ y
    want = np.array([_eps_soft(zj, lam, EPS) for zj in z])
    np.testing.assert_allclose(r.beta, want, rtol=1e-9, atol=1e-12)
    # and the eps -> 0 limit is soft-thresholding (eq. of the soft-threshold relation)
    soft = np.sign(z) * np.maximum(np.abs(z) - lam, 0.0)
    assert np.max(np.abs(r.beta - soft)) <= math.sqrt(EPS * np.max(np.abs(z))) + 1e-9


# --------------------------------------------------------------------------
# Two-variable FLSA (X = I, p = 2, one edge): optimality conditions, then soft-thresholding
# --------------------------------------------------------------------------
def _flsa2(y1, y2, l1, l2):
    if abs(y1 - y2) <= 2 * l2:
        b = np.array([(y1 + y2) / 2, (y1 + y2) / 2])
    else:
        s = math.copysign(1.0, y1 - y2)
        b = np.array([y1 - l2 * s, y2 + l2 * s])
    return np.sign(b) * np.maximum(np.abs(b) - l1, 0.0)


@pytest.mark.parametrize("y1,y2,l1,l2", [(3.0, 1.0, 0.0, 0.4), (3.0, 1.0, 0.0, 1.6), (-2.0, 1.5, 0.5, 0.3),
                                          (2.0, 2.5, 0.7, 0.6), (0.4, -0.3, 1.0, 0.1), (5.0, -4.0, 0.2, 2.0)])
def test_two_variable_flsa(y1, y2, l1, l2):
    P = _problem(np.eye(2), [y1, y2], [[0, 1]])
    r = oracle.solve(P, l1, l2, tol=0.0, max_iter=4000, inner_tol=1e-14)
    want = _flsa2(y1, y2, l1, l2)
    np.testing.assert_allclose(r.beta, want, atol=5e-6)
    assert oracle.objective(P, l1, l2, r.beta) - oracle.objective(P, l1, l2, want) <= 1e-6


# --------------------------------------------------------------------------
# Soft-threshold relation for the FLSA on any graph: b(l1, l2) = soft(b(0, l2), l1)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("graph", ["chain", "lattice"])
def test_soft_threshold_relation(graph):
    p = 6 if graph == "chain" else 9
    edges = flrgen.chain_edges(p) if graph == "chain" else flrgen.lattice_edges(3)
    y = np.array([3.0, 3.2, -1.0, -1.4, 0.5, 4.0, 2.0, -2.5, 0.1][:p])
    P = _problem(np.eye(p), y, edges)
    l2 = 0.25
    b0 = oracle.solve(P, 0.0, l2, tol=0.0, max_iter=6000).beta
    l1 = 0.8
    # keep every coordinate away from the threshold so the eps perturbation stays small
    assert np.min(np.abs(np.abs(b0) - l1)) > 0.05
    b1 = oracle.solve(P, l1, l2, tol=0.0, max_iter=6000).beta
    np.testing.assert_allclose(b1, np.sign(b0) * np.maximum(np.abs(b0) - l1, 0.0), atol=5e-6)


# --------------------------------------------------------------------------
# Lemma 2: f_eps decreases monotonically along the MM iterates (also with inexact PCG)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("method,inner", [(oracle.ALG1, 0.0), (oracle.ALG2, 1e-4), (oracle.ALG2, 1e-10)])
@pytest.mark.parametrize("graph", ["chain", "lattice"])
def test_monotone_descent(method, inner, graph):
    inst = flrgen.small_instance(30, 64, graph, seed=7, lam1=0.2, lam2=0.6)
    P = oracle.Problem.from_instance(inst)
    r = oracle.solve(P, inst.lam1, inst.lam2, tol=1e-10, inner_tol=inner, method=method, trajectory=True,
                     max_iter=400)
    fe = np.concatenate([[oracle.objective_eps(P, inst.lam1, inst.lam2, EPS, oracle.init_beta(P))], r.traj["f_eps"]])
    assert np.all(np.diff(fe) <= 1e-13 * np.abs(fe[:-1]))
    assert len(fe) > 5


# --------------------------------------------------------------------------
# Brute-force QP on tiny problems: enumerate sign patterns of b_j and of b_j - b_k;
# on each face the objective is a quadratic whose minimizer is a candidate; f* = min f over candidates
# --------------------------------------------------------------------------
def _groups(p, edges, fused):
    parent = list(range(p))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for (j, k), f in zip(edges, fused):
        if f:
            parent[find(j)] = find(k)
    roots = sorted({find(j) for j in range(p)})
    return np.array([roots.index(find(j)) for j in range(p)]), len(roots)


def brute_force_min(X, y, edges, l1, l2):
    n, p = X.shape
    m = len(edges)
    D = np.zeros((m, p))
    for e, (j, k) in enumerate(edges):
        D[e, j], D[e, k] = 1.0, -1.0
    best = math.inf
    best_b = None
    XtX, Xty = X.T @ X, X.T @ y

    def f(b):
        return 0.5 * np.sum((y - X @ b) ** 2) + l1 * np.abs(b).sum() + l2 * np.abs(D @ b).sum()

    for tau in itertools.product((-1, 0, 1), repeat=m):
        gid, G = _groups(p, edges, [t == 0 for t in tau])
        lin_e = l2 * (D.T @ np.array(tau, dtype=float)) if m else np.zeros(p)
        for sig in itertools.product((-1, 0, 1), repeat=G):
            free = [g for g in range(G) if sig[g] != 0]
            T = np.zeros((p, len(free)))
            sj = np.zeros(p)
            for col, g in enumerate(free):
                T[gid == g, col] = 1.0
                sj[gid == g] = sig[g]
            if T.shape[1] == 0:
                b = np.zeros(p)
            else:
                H = T.T @ XtX @ T
                rhs = T.T @ (Xty - l1 * sj - lin_e)
                b = T @ np.linalg.solve(H, rhs)
            v = f(b)
            if v < best:
                best, best_b = v, b
    return best, best_b


@pytest.mark.parametrize("graph,p", [("chain", 5), ("lattice", 4), ("allpairs", 4)])
def test_brute_force_qp(graph, p):
    rng = np.random.default_rng(11)
    n = p + 3
    X = rng.standard_normal((n, p))
    edges = {"chain": flrgen.chain_edges(p), "lattice": flrgen.lattice_edges(2), "allpairs": flrgen.all_pairs_edges(p)}[graph]
    beta_t = np.array([1.0, 1.0, 0.0, -0.5, -0.5][:p])
    y = X @ beta_t + 0.3 * rng.standard_normal(n)
    l1, l2 = 0.4, 0.7
    fstar, bstar = brute_force_min(X, y, [tuple(e) for e in edges], l1, l2)
    P = _problem(X, y, edges)
    r = oracle.solve(P, l1, l2, tol=0.0, max_iter=3000, inner_tol=1e-14)
    f_mm = oracle.objective(P, l1, l2, r.beta)
    # the MM iterate minimizes f_eps; its excess over min f is O((p+m) * lambda * eps * log(1/eps))
    assert f_mm >= fstar - 1e-12 * fstar
    assert f_mm - fstar <= 1e-6 * max(1.0, fstar)
    np.testing.assert_allclose(r.beta, bstar, atol=1e-4)


# --------------------------------------------------------------------------
# Stationarity (Lemma 2): at the MM limit, grad f_eps = 0, i.e. Q(b) b = c
# --------------------------------------------------------------------------
@pytest.mark.parametrize("graph", ["chain", "lattice"])
def test_stationary_at_convergence(graph):
    inst = flrgen.small_instance(25, 36, graph, seed=9, lam1=0.3, lam2=0.5)
    P = oracle.Problem.from_instance(inst)
    r = oracle.solve(P, inst.lam1, inst.lam2, tol=0.0, max_iter=4000, inner_tol=1e-14, method=oracle.ALG1)
    g = oracle.gradient_eps(P, inst.lam1, inst.lam2, EPS, r.beta)
    c = oracle.system(P, inst.lam1, inst.lam2, EPS, r.beta)[1]
    assert np.max(np.abs(g)) <= 1e-6 * np.max(np.abs(c))


# --------------------------------------------------------------------------
# Algorithm 1 (dense Cholesky) and Algorithm 2 (PCG) follow one MM trajectory
# --------------------------------------------------------------------------
@pytest.mark.parametrize("graph", ["chain", "lattice"])
def test_alg1_alg2_agree(graph):
    inst = flrgen.small_instance(40, 100, graph, seed=12, lam1=0.1, lam2=0.5)
    P = oracle.Problem.from_instance(inst)
    r1 = oracle.solve(P, inst.lam1, inst.lam2, tol=1e-8, method=oracle.ALG1)
    r2 = oracle.solve(P, inst.lam1, inst.lam2, tol=1e-8, inner_tol=1e-13, method=oracle.ALG2)
    assert r1.status == r2.status == oracle.OK
    assert r1.mm_iters == r2.mm_iters
    assert np.max(np.abs(r1.beta - r2.beta)) <= 1e-7 * np.max(np.abs(r1.beta))
    assert abs(r1.objective - r2.objective) <= 1e-11 * r1.objective


def test_status_codes():
    inst = flrgen.small_instance(20, 30, "chain", seed=1)
    P = oracle.Problem.from_instance(inst)
    r = oracle.solve(P, 0.1, 0.5, tol=1e-12, max_iter=2)
    assert r.status == oracle.MAX_ITER and r.mm_iters == 2
    r = oracle.solve(P, -0.1, 0.5)
    assert r.status == oracle.BAD_ARG


def test_bf16_rounding_ties_to_even():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties to even -> 1.0
    # 1 + 3*2^-9 is above the tie -> 1 + 2^-7 ; a value a hair above a tie must round up
    vals = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 1.0 + 2.0 ** -8 + 2.0 ** -40, -(1.0 + 2.0 ** -8 + 2.0 ** -40)])
    got = flrgen.bf16_bits_to_f64(flrgen.f64_to_bf16_bits(vals))
    np.testing.assert_array_equal(got, [1.0, 1.0 + 2.0 ** -7, 1.0 + 2.0 ** -7, -(1.0 + 2.0 ** -7)])
