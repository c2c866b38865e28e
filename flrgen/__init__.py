"""Seeded synthetic workloads for fused lasso regression (FLR).

This module only draws inputs: design matrices X, responses y, edge sets E
and the (lambda1, lambda2) settings.  It holds none of the solver's
arithmetic, so both the FP64 CPU oracle (under ``oracle/``) and the HIP
path can be fed from it without sharing any of the method's code.

Data model (section 5, the generating equation of the numerical studies):
y = X beta_true + sigma * noise with rows of X drawn from a Gaussian.
The graph families follow the introduction: the chain of the standard FLR,
the q x q lattice of the two-dimensional FLR, and the all-pairs set of the
clustered / pairwise fused lasso.  Lattice coefficients are vec(B), i.e.
column-major: index(i, j) = i + q * j (section 5.2, scenario C4).

Every array is drawn from numpy's PCG64 through a SeedSequence that is
spawned into independent streams (beta, X, noise), so the same seed gives
the same instance on every machine.  X is generated in FP64 and then
rounded to its storage type; the stored values define the instance.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

F64, F32, BF16 = 0, 1, 2
DTYPE_NAMES = {F64: "f64", F32: "f32", BF16: "bf16"}


# ----------------------------------------------------------------------------
# storage rounding
# ----------------------------------------------------------------------------
def f64_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to bfloat16 (round-to-nearest-even) and return the
    16-bit patterns as uint16.

    A direct FP64 -> FP32 -> BF16 chain can round twice; rounding to FP32
    with round-to-odd first (truncate, then set the last bit when inexact)
    keeps the second rounding correct because FP32 carries 16 spare bits.
    Inputs must be finite.
    """
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = x.astype(np.float32)
    back = f.astype(np.float64)
    inexact = back != x
    # step toward zero where round-to-nearest went away from zero
    away = inexact & (np.abs(back) > np.abs(x))
    f = np.where(away, np.nextafter(f, np.float32(0.0)), f)
    bits = f.view(np.uint32).copy()
    bits[inexact] |= np.uint32(1)
    lsb = (bits >> np.uint32(16)) & np.uint32(1)
    bits = bits + np.uint32(0x7FFF) + lsb
    return (bits >> np.uint32(16)).astype(np.uint16)


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    """Exact widening of bfloat16 bit patterns to FP64."""
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def store(x64: np.ndarray, dtype: int) -> np.ndarray:
    """Round an FP64 matrix to its storage type (f64 copy, f32, or bf16 bits)."""
    if dtype == F64:
        return np.ascontiguousarray(x64, dtype=np.float64)
    if dtype == F32:
        return np.ascontiguousarray(x64.astype(np.float32))
    if dtype == BF16:
        return f64_to_bf16_bits(x64)
    raise ValueError(f"unknown dtype {dtype}")


def widen(xs: np.ndarray, dtype: int) -> np.ndarray:
    """Exact FP64 view of a stored matrix."""
    if dtype == BF16:
        return bf16_bits_to_f64(xs)
    return np.asarray(xs, dtype=np.float64)


# ----------------------------------------------------------------------------
# edge sets
# ----------------------------------------------------------------------------
def chain_edges(p: int) -> np.ndarray:
    """Chain graph of the standard FLR: pairs (j-1, j), 0-based."""
    j = np.arange(1, p, dtype=np.int64)
    return np.stack([j - 1, j], axis=1) if p > 1 else np.zeros((0, 2), np.int64)


def lattice_edges(q: int) -> np.ndarray:
    """q x q lattice with column-major vectorisation index(i, j) = i + q*j.

    Vertical neighbours (i-1, j)-(i, j) are index-adjacent; horizontal
    neighbours (i, j-1)-(i, j) are q apart.  m = 2 q (q - 1).
    """
    ii, jj = np.meshgrid(np.arange(q, dtype=np.int64), np.arange(q, dtype=np.int64), indexing="ij")
    idx = ii + q * jj
    vert = np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], axis=1)
    horz = np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], axis=1)
    e = np.concatenate([vert, horz], axis=0)
    return e[np.lexsort((e[:, 1], e[:, 0]))]


def all_pairs_edges(p: int) -> np.ndarray:
    """All unordered pairs (j, k), j < k (clustered / pairwise fused lasso)."""
    j, k = np.triu_indices(p, 1)
    return np.stack([j.astype(np.int64), k.astype(np.int64)], axis=1)


# ----------------------------------------------------------------------------
# true coefficient patterns
# ----------------------------------------------------------------------------
def piecewise_beta(p: int, nblocks: int, zero_frac: float, rng: np.random.Generator,
                   lo: float = -2.0, hi: float = 2.0) -> np.ndarray:
    """Piecewise-constant beta: nblocks equal blocks, round(zero_frac*nblocks)
    of them zero (chosen at random), the rest at levels drawn U[lo, hi]."""
    edges = np.linspace(0, p, nblocks + 1).round().astype(np.int64)
    nzero = int(round(zero_frac * nblocks))
    zero = np.zeros(nblocks, dtype=bool)
    zero[rng.choice(nblocks, size=nzero, replace=False)] = True
    levels = rng.uniform(lo, hi, size=nblocks)
    beta = np.zeros(p)
    for b in range(nblocks):
        if not zero[b]:
            beta[edges[b]:edges[b + 1]] = levels[b]
    return beta


def rectangles_beta(q: int, nrect: int, rng: np.random.Generator) -> np.ndarray:
    """q x q image of nrect axis-aligned constant rectangles on a zero
    background (later rectangles overwrite earlier ones), returned as vec(B)
    in column-major order.  Side lengths U{q/10 .. 3q/10}, levels U[-2, 2]
    with |level| >= 0.5."""
    img = np.zeros((q, q))
    smin = max(1, q // 10)
    smax = max(smin, (3 * q) // 10)
    for _ in range(nrect):
        h = int(rng.integers(smin, smax + 1))
        w = int(rng.integers(smin, smax + 1))
        i0 = int(rng.integers(0, q - h + 1))
        j0 = int(rng.integers(0, q - w + 1))
        lev = 0.0
        while abs(lev) < 0.5:
            lev = float(rng.uniform(-2.0, 2.0))
        img[i0:i0 + h, j0:j0 + w] = lev
    return img.ravel(order="F").copy()


def cluster_beta(p: int, nclust: int, rng: np.random.Generator) -> np.ndarray:
    """nclust equal-valued random clusters (values U[-2, 2]) over a zero
    background covering half of the coordinates."""
    beta = np.zeros(p)
    idx = rng.permutation(p)[: p // 2]
    labels = rng.integers(0, nclust, size=idx.size)
    levels = rng.uniform(-2.0, 2.0, size=nclust)
    beta[idx] = levels[labels]
    return beta


# ----------------------------------------------------------------------------
# design matrices (generated in FP64, rounded to storage type)
# ----------------------------------------------------------------------------
def gaussian_x(n: int, p: int, rng: np.random.Generator, dtype: int, chunk_rows: int = 512) -> np.ndarray:
    """Rows iid N(0, I_p), drawn chunk by chunk and rounded to dtype."""
    out_dt = {F64: np.float64, F32: np.float32, BF16: np.uint16}[dtype]
    out = np.empty((n, p), dtype=out_dt)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        out[r0:r1] = store(rng.standard_normal((r1 - r0, p)), dtype)
    return out


def ar1_x(n: int, p: int, rho: float, rng: np.random.Generator, dtype: int) -> np.ndarray:
    """Rows iid AR(1) along the column index with unit marginal variance:
    X[i,0] = z, X[i,j] = rho X[i,j-1] + sqrt(1-rho^2) z."""
    z = rng.standard_normal((n, p))
    s = math.sqrt(1.0 - rho * rho)
    x = np.empty((n, p))
    x[:, 0] = z[:, 0]
    for j in range(1, p):
        x[:, j] = rho * x[:, j - 1] + s * z[:, j]
    return store(x, dtype)


def matvec_rows(xs: np.ndarray, dtype: int, v: np.ndarray, chunk_rows: int = 256) -> np.ndarray:
    """FP64 X v for the data model y = X beta + noise (chunked widening).

    Each row is summed by numpy's own pairwise reduction rather than a BLAS
    product, whose summation order depends on its thread count: the same
    seed must give bitwise the same y on every machine."""
    n = xs.shape[0]
    out = np.empty(n)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        out[r0:r1] = np.add.reduce(widen(xs[r0:r1], dtype) * v[None, :], axis=1)
    return out


# ----------------------------------------------------------------------------
# problem instances
# ----------------------------------------------------------------------------
@dataclass
class Instance:
    name: str
    X: np.ndarray            # stored matrix (float64, float32 or uint16 bf16 bits), row-major n x p
    dtype: int
    y: np.ndarray            # float64, length n
    edges: np.ndarray        # int64 (m, 2), 0-based, j < k
    beta_true: np.ndarray
    lam1: float = 0.1
    lam2: float = 0.1
    eps: float = 1e-8
    tol: float = 1e-8
    graph: str = "chain"
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def p(self) -> int:
        return int(self.X.shape[1])

    @property
    def m(self) -> int:
        return int(self.edges.shape[0])


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]


def make_instance(name, n, p, graph, dtype, beta_fn, xfn, sigma, seed, lam1, lam2,
                  eps=1e-8, tol=1e-8, q=None, y_f32=False) -> Instance:
    rb, rx, rn = _streams(seed)
    if graph == "chain":
        edges = chain_edges(p)
    elif graph == "lattice":
        assert q is not None and q * q == p
        edges = lattice_edges(q)
    elif graph == "allpairs":
        edges = all_pairs_edges(p)
    elif graph == "none":
        edges = np.zeros((0, 2), np.int64)
    else:
        raise ValueError(graph)
    beta = beta_fn(rb)
    X = xfn(rx)
    y = matvec_rows(X, dtype, beta) + sigma * rn.standard_normal(n)
    if y_f32:
        y = y.astype(np.float32).astype(np.float64)
    return Instance(name=name, X=X, dtype=dtype, y=y, edges=edges, beta_true=beta, lam1=lam1, lam2=lam2,
                    eps=eps, tol=tol, graph=graph, meta={"seed": seed, "sigma": sigma, "q": q})


def config1(seed: int = 1, n: int = 100, p: int = 500) -> Instance:
    """Standard FLR, n=100, p=500, FP64 X iid N(0,1); beta 10 blocks, half
    zero, levels U[-2,2]; unit noise; (lambda1, lambda2) = (0.1, 0.5)."""
    return make_instance("c1_chain_n%d_p%d_f64" % (n, p), n, p, "chain", F64,
                         lambda r: piecewise_beta(p, 10, 0.5, r),
                         lambda r: gaussian_x(n, p, r, F64), 1.0, seed, 0.1, 0.5)


def config2(seed: int = 2, n: int = 1000, p: int = 10000, dtype: int = F32) -> Instance:
    """Standard FLR, n=1000, p=10000, X FP32 rows AR(1) rho=0.5; beta 50
    blocks, 80% zero; noise sigma 0.5; (lambda1, lambda2) = (0.5, 1.0)."""
    nb = max(1, min(50, p // 4))
    return make_instance("c2_chain_ar1_n%d_p%d_%s" % (n, p, DTYPE_NAMES[dtype]), n, p, "chain", dtype,
                         lambda r: piecewise_beta(p, nb, 0.8, r),
                         lambda r: ar1_x(n, p, 0.5, r, dtype), 0.5, seed, 0.5, 1.0)


GRID16 = np.logspace(-2.0, 1.0, 16)


def config3(seed: int = 3, q: int = 100, n: int = 2000) -> Instance:
    """Two-dimensional FLR on a q x q lattice (p = q^2), n=2000, X FP32 iid
    N(0,1); beta a q x q image of 5 rectangles; unit noise.  The lambda grid
    is the 16 x 16 log-spaced grid over [0.01, 10]^2 (GRID16)."""
    p = q * q
    inst = make_instance("c3_lattice_q%d_n%d_f32" % (q, n), n, p, "lattice", F32,
                         lambda r: rectangles_beta(q, 5, r),
                         lambda r: gaussian_x(n, p, r, F32), 1.0, seed, 0.1, 0.1, q=q)
    return inst


def grid_lambdas(values=GRID16):
    """All (lambda1, lambda2) pairs of a square grid, lambda1 major."""
    l1, l2 = np.meshgrid(values, values, indexing="ij")
    return l1.ravel().copy(), l2.ravel().copy()


def config4(seed: int = 4, n: int = 5000, p: int = 50000) -> Instance:
    """Large standard FLR, n=5000, p=50000, X stored BF16 (drawn N(0,1) in
    FP64, rounded), y rounded to FP32; beta 200 blocks, 90% zero; unit
    noise; (lambda1, lambda2) = (0.5, 1.0)."""
    nb = max(1, min(200, p // 4))
    return make_instance("c4_chain_n%d_p%d_bf16" % (n, p), n, p, "chain", BF16,
                         lambda r: piecewise_beta(p, nb, 0.9, r),
                         lambda r: gaussian_x(n, p, r, BF16), 1.0, seed, 0.5, 1.0, y_f32=True)


SERVE_PS = (1000, 5000, 10000, 50000)


def serving_cell(p_nominal: int, graph: str, seed: int, scale: float = 1.0) -> Instance:
    """One resident problem of the serving mix: n = p/5, X FP32 N(0,1).
    chain: beta as config 1 (10 blocks, half zero); lattice: q=round(sqrt(p)),
    p := q^2, beta 5 rectangles; allpairs (p <= 1000): 5 clusters.
    ``scale`` < 1 shrinks p for tests."""
    p_nom = max(8, int(round(p_nominal * scale)))
    if graph == "lattice":
        q = int(round(math.sqrt(p_nom)))
        p = q * q
        n = max(2, p // 5)
        return make_instance("serve_lattice_q%d" % q, n, p, "lattice", F32,
                             lambda r: rectangles_beta(q, 5, r),
                             lambda r: gaussian_x(n, p, r, F32), 1.0, seed, 0.1, 0.1, q=q)
    p = p_nom
    n = max(2, p // 5)
    if graph == "chain":
        return make_instance("serve_chain_p%d" % p, n, p, "chain", F32,
                             lambda r: piecewise_beta(p, 10, 0.5, r),
                             lambda r: gaussian_x(n, p, r, F32), 1.0, seed, 0.1, 0.1)
    if graph == "allpairs":
        return make_instance("serve_allpairs_p%d" % p, n, p, "allpairs", F32,
                             lambda r: cluster_beta(p, 5, r),
                             lambda r: gaussian_x(n, p, r, F32), 1.0, seed, 0.1, 0.1)
    raise ValueError(graph)


def serving_requests(nreq: int, seed: int = 5, rate: float = 1.0, ps=SERVE_PS):
    """Request stream of the serving mix: Poisson arrivals at ``rate`` per
    second, p uniform over ``ps``, graph uniform over the types allowed for
    that p (all-pairs only for p <= 1000), (lambda1, lambda2) log-uniform in
    [0.01, 10]^2, and an instance slot in 0..3 (4 resident problems per cell)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, size=nreq))
    out = []
    for i in range(nreq):
        p = int(ps[int(rng.integers(0, len(ps)))])
        kinds = ["chain", "lattice"] + (["allpairs"] if p <= 1000 else [])
        g = kinds[int(rng.integers(0, len(kinds)))]
        l1 = float(10.0 ** rng.uniform(-2.0, 1.0))
        l2 = float(10.0 ** rng.uniform(-2.0, 1.0))
        slot = int(rng.integers(0, 4))
        out.append({"t": float(t[i]), "p": p, "graph": g, "lam1": l1, "lam2": l2, "slot": slot})
    return out


# ----------------------------------------------------------------------------
# the paper's simulation scenarios: section 5.1 (C1-C3, chain) and 5.2 (C4, lattice)
# ----------------------------------------------------------------------------
PAPER_LAMBDAS = ((0.1, 0.1), (0.1, 1.0), (1.0, 0.1), (1.0, 1.0))  # both sections' four settings
PAPER_TOL = 1e-5     # relative objective change at which every algorithm stops (section 5)
PAPER_N = 1000
PAPER_SIZES = {"C1": (200, 1000, 10000, 20000), "C2": (200, 1000, 10000, 20000),
               "C3": (200, 1000, 10000, 20000), "C4": (16, 32, 64, 128)}  # p, or the lattice side q for C4
_PAPER_IDS = {"C1": 1, "C2": 2, "C3": 3, "C4": 4}


def paper_beta(scenario: str, size: int) -> np.ndarray:
    """True coefficients of the scenario (section 5.1 for C1-C3, indices
    there are 1-based; section 5.2 for C4, where size is the side q and beta =
    vec(B) of the q x q block pattern)."""
    if scenario == "C1":  # sparse: 41 nonzeros at fixed positions
        b = np.zeros(size)
        b[0:20] = 2.0
        b[120:125] = 2.0
        b[40] = 3.0
        b[70:85] = 1.0
        return b
    if scenario == "C2":  # moderately sparse: 30 % nonzero
        assert size % 10 == 0
        b = np.zeros(size)
        b[size // 10:2 * size // 10] = 1.0
        b[2 * size // 10:4 * size // 10] = 2.0
        return b
    if scenario == "C3":  # dense: +1 on the first half, -1 on the second
        assert size % 2 == 0
        return np.where(np.arange(size) < size // 2, 1.0, -1.0)
    if scenario == "C4":  # q x q: +2 on the four diagonal blocks of side q/4, -2 on the anti-diagonal ones
        q = size
        assert q % 4 == 0
        h = q // 4
        B = np.zeros((q, q))
        for k in range(4):
            B[k * h:(k + 1) * h, k * h:(k + 1) * h] = 2.0
            B[k * h:(k + 1) * h, (3 - k) * h:(4 - k) * h] = -2.0
        return B.ravel(order="F").copy()
    raise ValueError(scenario)


def paper_scenario(scenario: str, size: int, dataset: int, n: int = PAPER_N) -> Instance:
    """Data set `dataset` (0..9 in the paper) of a scenario: X rows iid
    N(0, I_p) in FP64, y = X beta + N(0, I_n) (the generating equation of
    section 5.1), chain edges for C1-C3 and the q x q lattice for C4;
    tolerance 1e-5, eps 1e-8 (section 5).  lam1/lam2 hold the first of the
    four settings; a caller solves all four on the same data set."""
    p = size * size if scenario == "C4" else size
    graph = "lattice" if scenario == "C4" else "chain"
    seed = [1306, _PAPER_IDS[scenario], size, dataset]
    beta = paper_beta(scenario, size)
    l1, l2 = PAPER_LAMBDAS[0]
    return make_instance("paper_%s_%d_d%d" % (scenario, size, dataset), n, p, graph, F64, lambda r: beta,
                         lambda r: gaussian_x(n, p, r, F64), 1.0, seed, l1, l2, tol=PAPER_TOL,
                         q=size if scenario == "C4" else None)


def small_instance(n: int, p: int, graph: str = "chain", dtype: int = F64, seed: int = 11,
                   lam1: float = 0.1, lam2: float = 0.5, q=None, sigma: float = 1.0,
                   x_kind: str = "gauss") -> Instance:
    """Small instances for parity and unit tests (same families, any size)."""
    if graph == "lattice":
        q = q or int(round(math.sqrt(p)))
        p = q * q
        bfn = lambda r: rectangles_beta(q, 3, r)
    elif graph == "allpairs":
        bfn = lambda r: cluster_beta(p, 3, r)
    else:
        bfn = lambda r: piecewise_beta(p, max(1, min(10, p // 4)), 0.5, r)
    if x_kind == "ar1":
        xfn = lambda r: ar1_x(n, p, 0.5, r, dtype)
    else:
        xfn = lambda r: gaussian_x(n, p, r, dtype)
    return make_instance("small_%s_n%d_p%d_%s" % (graph, n, p, DTYPE_NAMES[dtype]), n, p, graph, dtype,
                         bfn, xfn, sigma, seed, lam1, lam2, q=q)
