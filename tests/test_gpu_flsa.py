"""The fused lasso signal approximation (X = I) through flr_create_flsa: no X
is stored, every product X^T X p is p.  Checked against closed forms (the
two-variable FLSA and the soft-threshold relation of the introduction),
against the oracle given an explicit identity X, against the general path
given the same identity X, on a chain and on a synthetic 2-D image (the
denoising setting of section 5.2, a q x q lattice of rectangles plus noise),
and through the batched grid."""
import math

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


def _flsa2(y1, y2, l1, l2):
    # optimality conditions of the two-variable FLSA, then soft-thresholding
    if abs(y1 - y2) <= 2 * l2:
        b = np.array([(y1 + y2) / 2, (y1 + y2) / 2])
    else:
        s = math.copysign(1.0, y1 - y2)
        b = np.array([y1 - l2 * s, y2 + l2 * s])
    return np.sign(b) * np.maximum(np.abs(b) - l1, 0.0)


@pytest.mark.parametrize("y1,y2,l1,l2", [(3.0, 1.0, 0.0, 0.4), (3.0, 1.0, 0.0, 1.6), (-2.0, 1.5, 0.5, 0.3),
                                          (2.0, 2.5, 0.7, 0.6), (5.0, -4.0, 0.2, 2.0)])
def test_two_variable_closed_form(flr, ctx, y1, y2, l1, l2):
    prob = flr.Problem.flsa(ctx, [y1, y2], [[0, 1]])
    assert flr.flr_problem_is_flsa(prob.h) == 1
    sol = prob.solve(l1, l2, tol=1e-15, inner_tol=1e-14, max_iter=4000)
    prob.close()
    want = _flsa2(y1, y2, l1, l2)
    print("  y=(%g,%g) lam=(%g,%g) beta=%s closed form %s mm=%d" % (y1, y2, l1, l2, sol.beta, want, sol.mm_iters))
    np.testing.assert_allclose(sol.beta, want, atol=5e-6)


def _chain_signal(p=300, seed=3):
    rng = np.random.default_rng(seed)
    beta = rng.uniform(-2, 2, 6)[np.minimum(np.arange(p) * 6 // p, 5)]
    return beta + 0.3 * rng.standard_normal(p)


def _oracle_identity(y, edges, l1, l2, **kw):
    p = y.size
    P = oracle.Problem(np.eye(p), oracle.F64, y, np.asarray(edges, dtype=np.int64).reshape(-1, 2))
    return oracle.solve(P, l1, l2, **kw)


@pytest.mark.parametrize("l1,l2", [(0.3, 0.7), (0.0, 0.7)])
def test_chain_matches_oracle_and_dense_identity(flr, ctx, l1, l2):
    y = _chain_signal()
    e = flrgen.chain_edges(y.size)
    kw = dict(tol=1e-8, inner_tol=INNER, max_cg=100 * y.size)
    prob = flr.Problem.flsa(ctx, y, e)
    sol = prob.solve(l1, l2, **kw)
    fp_flsa = prob.footprint
    prob.close()
    dense = flr.Problem(ctx, np.eye(y.size), flrgen.F64, y, e)
    sd = dense.solve(l1, l2, **kw)
    fp_dense = dense.footprint
    dense.close()
    ref = _oracle_identity(y, e, l1, l2, tol=1e-8, inner_tol=INNER, max_cg=100 * y.size)
    sc = np.max(np.abs(ref.beta))
    err, errd = np.max(np.abs(sol.beta - ref.beta)) / sc, np.max(np.abs(sol.beta - sd.beta)) / sc
    print("  lam=(%g,%g) flsa mm=%d cg=%d | dense X=I mm=%d | oracle mm=%d | err=%.2e vs dense %.2e" % (
        l1, l2, sol.mm_iters, sol.cg_iters, sd.mm_iters, ref.mm_iters, err, errd), flush=True)
    assert sol.status == flr.FLR_OK and sol.mm_iters == ref.mm_iters == sd.mm_iters
    assert err <= 1e-8 and errd <= 1e-8
    assert abs(sol.objective - ref.objective) <= 1e-11 * ref.objective
    assert fp_flsa < fp_dense  # no X on the device


def test_soft_threshold_relation(flr, ctx):
    # introduction: for X = I on any graph, b(lambda1, lambda2) = soft(b(0, lambda2), lambda1)
    y = _chain_signal(p=240, seed=5)
    e = flrgen.chain_edges(y.size)
    prob = flr.Problem.flsa(ctx, y, e)
    b0 = prob.solve(0.0, 0.5, tol=1e-14, inner_tol=1e-14, max_iter=8000, max_cg=100 * y.size).beta
    l1 = 0.6
    assert np.min(np.abs(np.abs(b0) - l1)) > 0.02
    b1 = prob.solve(l1, 0.5, tol=1e-14, inner_tol=1e-14, max_iter=8000, max_cg=100 * y.size).beta
    prob.close()
    np.testing.assert_allclose(b1, np.sign(b0) * np.maximum(np.abs(b0) - l1, 0.0), atol=5e-6)


def test_image_denoising_lattice(flr, ctx):
    # a 40 x 40 image of rectangles plus noise, the 2-D FLSA on the lattice (banded M, bandwidth 40)
    q = 40
    rng = np.random.default_rng(9)
    img = flrgen.rectangles_beta(q, 5, rng)
    y = img + 0.5 * rng.standard_normal(q * q)
    e = flrgen.lattice_edges(q)
    prob = flr.Problem.flsa(ctx, y, e)
    sol = prob.solve(0.05, 0.4, tol=1e-8, inner_tol=INNER)
    prob.close()
    ref = _oracle_identity(y, e, 0.05, 0.4, tol=1e-8, inner_tol=INNER, method=oracle.ALG2)
    err = np.max(np.abs(sol.beta - ref.beta)) / np.max(np.abs(ref.beta))
    mse_noisy, mse_fit = np.mean((y - img) ** 2), np.mean((sol.beta - img) ** 2)
    print("  denoising q=%d mm=%d (oracle %d) err=%.2e  mse noisy %.3f -> fit %.3f" % (
        q, sol.mm_iters, ref.mm_iters, err, mse_noisy, mse_fit), flush=True)
    assert sol.status == flr.FLR_OK and sol.mm_iters == ref.mm_iters
    assert err <= 1e-8
    assert mse_fit < 0.5 * mse_noisy  # the fused fit removes most of the noise


def test_grid_on_flsa(flr, ctx):
    y = _chain_signal(p=200, seed=7)
    e = flrgen.chain_edges(y.size)
    l1 = np.array([0.1, 0.3, 0.0])
    l2 = np.array([0.5, 0.2, 0.8])
    prob = flr.Problem.flsa(ctx, y, e)
    st, beta, res = prob.solve_grid(l1, l2, tol=1e-8, inner_tol=INNER, max_cg=100 * y.size)
    singles = [prob.solve(a, b, tol=1e-8, inner_tol=INNER, max_cg=100 * y.size) for a, b in zip(l1, l2)]
    prob.close()
    for b in range(l1.size):
        err = np.max(np.abs(beta[b] - singles[b].beta)) / np.max(np.abs(singles[b].beta))
        assert res[b]["status"] == flr.FLR_OK and res[b]["mm_iters"] == singles[b].mm_iters
        assert err <= 1e-8
