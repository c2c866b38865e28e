"""Autotuner for the launch shapes of the two streaming kernels.

The row-panel kernel (X v) and the column-panel kernel (X^T u) split X into
tiles; how many workgroups each launch gets (hence rows per tile) is a
trade-off between filling 256 CUs, the per-workgroup latency chain and the
partial sums the next launch has to add.  For a problem shape (n, p, dtype)
this times candidate workgroup targets with the library's own HIP-event
profiler and caches the fastest in a JSON file (``$FLR_TUNE_CACHE``, default
``~/.cache/flr_tune.json``).  ``Problem`` consults the cache at creation, then
the shapes shipped with the package (``tuned_gfx950.json``, measured on an
MI355X for the benchmark workloads); without either the engine's default of
512 workgroups per launch applies.
"""
from __future__ import annotations

import contextlib
import json
import os

CANDIDATES = (256, 384, 512, 768, 1024, 2048)
_ENV_A, _ENV_B = "FLR_TARGET_WG_A", "FLR_TARGET_WG_B"


def cache_path() -> str:
    return os.environ.get("FLR_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "flr_tune.json"))


def _key(n, p, dtype) -> str:
    return "gfx950:n=%d:p=%d:dtype=%d" % (n, p, dtype)


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")


def _read(path) -> dict:
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def load() -> dict:
    """The user's tuning cache (entries measured on this machine)."""
    return _read(cache_path())


def load_shipped() -> dict:
    """Tuned shapes that ship with the package."""
    return _read(SHIPPED)


def lookup(n, p, dtype):
    """Tuned shapes for this problem shape: the user's cache first, then the shipped entries."""
    k = _key(n, p, dtype)
    return load().get(k) or load_shipped().get(k)


def store(n, p, dtype, entry, path=None):
    """Add or replace one entry of the cache file (atomic rewrite)."""
    path = path or cache_path()
    data = _read(path)
    data[_key(n, p, dtype)] = entry
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


@contextlib.contextmanager
def launch_shape(target_a=None, target_b=None):
    """Environment the engine reads at flr_create for the tile shapes."""
    old = {k: os.environ.get(k) for k in (_ENV_A, _ENV_B)}
    try:
        if target_a:
            os.environ[_ENV_A] = str(int(target_a))
        if target_b:
            os.environ[_ENV_B] = str(int(target_b))
        yield
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def tune(ctx, X, dtype, y, edges, lam1=0.5, lam2=1.0, candidates=CANDIDATES, reps=50, save=True, log=None):
    """Time each candidate for both kernels on this problem and cache the best."""
    from . import Problem, flr_profile_kernels

    n, p = int(X.shape[0]), int(X.shape[1])
    best = {"a": None, "b": None}
    times = {"a": {}, "b": {}}
    for cand in candidates:
        with launch_shape(cand, cand):
            prob = Problem(ctx, X, dtype, y, edges, use_tuned=False)
        prob.solve(lam1, lam2, tol=1e-6, max_iter=2)
        a_us, b_us, _ = flr_profile_kernels(prob.h, reps)
        prob.close()
        times["a"][cand] = a_us
        times["b"][cand] = b_us
        if log:
            log("autotune n=%d p=%d target=%d: A %.2f us, B %.2f us" % (n, p, cand, a_us, b_us))
    best["a"] = min(times["a"], key=times["a"].get)
    best["b"] = min(times["b"], key=times["b"].get)
    entry = {"target_wg_a": best["a"], "target_wg_b": best["b"], "a_us": times["a"][best["a"]],
             "b_us": times["b"][best["b"]], "times": {k: {str(c): t for c, t in v.items()} for k, v in times.items()}}
    if save:
        store(n, p, dtype, entry)
    return entry


def main(argv=None):
    """Tune the benchmark workloads on this GPU and write the entries to a
    cache file (``--out``; the package's shipped file by default)."""
    import argparse
    import sys

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--workload", action="append", choices=["c1", "c2", "c4"], default=None)
    ap.add_argument("--out", default=SHIPPED)
    ap.add_argument("--reps", type=int, default=50)
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import flrgen

    from . import Context

    makers = {"c1": flrgen.config1, "c2": flrgen.config2, "c4": flrgen.config4}
    ctx = Context(0)
    for w in args.workload or ["c2"]:
        inst = makers[w]()
        entry = tune(ctx, inst.X, inst.dtype, inst.y, inst.edges, inst.lam1, inst.lam2, reps=args.reps, save=False,
                     log=lambda m: print(m, flush=True))
        store(inst.n, inst.p, inst.dtype, entry, path=args.out)
        print("%s: target_wg_a=%d target_wg_b=%d" % (w, entry["target_wg_a"], entry["target_wg_b"]), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
