"""flr_solve_grid_static: the grid solve with its workspace in the library's
static device array.  Called through the C ABI and compared with
flr_solve_grid on the same problem and lambdas: the two run the same kernels
with the same arithmetic, so their results must be bitwise equal.  Two calls
in a row, the second on a smaller problem with fewer columns (the array keeps
the first call's contents), then the size limits."""
import numpy as np
import pytest

import flrgen

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


def _both(flr, ctx, inst, l1, l2, tol, **kw):
    prob = flr.Problem.from_instance(ctx, inst)
    fp0 = prob.footprint
    st_s, beta_s, res_s = prob.solve_grid(l1, l2, tol=tol, static=True, **kw)
    assert prob.footprint == fp0  # the static workspace is not the handle's
    st_a, beta_a, res_a = prob.solve_grid(l1, l2, tol=tol, **kw)
    prob.close()
    return (st_s, beta_s, res_s), (st_a, beta_a, res_a)


def _same(flr, s, a):
    st_s, beta_s, res_s = s
    st_a, beta_a, res_a = a
    assert st_s == st_a
    for rs, ra in zip(res_s, res_a):
        assert rs["status"] == ra["status"]
        assert rs["mm_iters"] == ra["mm_iters"] and rs["cg_iters"] == ra["cg_iters"]
        assert rs["objective"] == ra["objective"]
    assert np.array_equal(beta_s, beta_a)


def test_static_grid_two_calls_match_allocating_grid(flr, ctx):
    # first call: banded lattice columns (band factors in the array), six columns
    big = flrgen.small_instance(60, 400, "lattice", dtype=flrgen.F32, seed=71)
    l1 = np.array([0.05, 0.2, 0.6, 0.1, 1.0, 0.3])
    l2 = np.array([0.1, 0.3, 0.2, 0.8, 0.5, 0.05])
    print("static grid call 1: %s B=%d" % (big.name, l1.size), flush=True)
    s, a = _both(flr, ctx, big, l1, l2, 1e-7, inner_tol=1e-12)
    _same(flr, s, a)
    assert all(r["status"] == flr.FLR_OK for r in s[2])
    # second call: a smaller chain problem, fewer columns, one with lambda1 = 0 (Jacobi)
    small = flrgen.small_instance(30, 150, "chain", dtype=flrgen.F64, seed=72)
    l1 = np.array([0.0, 0.4, 0.1])
    l2 = np.array([0.5, 0.2, 0.9])
    print("static grid call 2: %s B=%d" % (small.name, l1.size), flush=True)
    s, a = _both(flr, ctx, small, l1, l2, 1e-7, inner_tol=1e-12, max_cg=50 * small.p)
    _same(flr, s, a)
    assert all(r["status"] == flr.FLR_OK for r in s[2])


def test_static_grid_rejects_sizes_beyond_the_array(flr, ctx):
    inst = flrgen.small_instance(20, 100, "chain", dtype=flrgen.F64, seed=73)
    prob = flr.Problem.from_instance(ctx, inst)
    too_many = np.full(300, 0.1)
    with pytest.raises(flr.FlrError) as ei:
        prob.solve_grid(too_many, too_many, tol=1e-6, static=True)
    assert ei.value.status == flr.FLR_ERR_INVALID_ARG
    prob.close()
    # a workspace larger than the array: 256 columns of p = 10^4
    wide = flrgen.small_instance(8, 10000, "chain", dtype=flrgen.F32, seed=74)
    prob = flr.Problem.from_instance(ctx, wide)
    cols = np.full(256, 0.1)
    with pytest.raises(flr.FlrError) as ei:
        prob.solve_grid(cols, cols, tol=1e-6, static=True)
    assert ei.value.status == flr.FLR_ERR_INVALID_ARG
    assert "bytes" in str(ei.value)
    prob.close()
