"""Build (or load from a cache) the base set and index of a named workload.

The benchmark and the full-size parity tests use this one recipe so that they
search the same index: the workload's base set from ``make_base``, then
``build_index`` with 20 Lloyd iterations and the workload's grid, metric and
integer mode.  The cache holds plain arrays (``numpy.savez``; loaded without
pickle) keyed by the workload's name, size, list count, subspaces and seed.
"""
from __future__ import annotations

import os
import time

import numpy as np

from .ivfpq import build_index
from .synth import WORKLOADS, make_base

DEFAULT_CACHE = "/tmp/amp_bench_cache"


def load_or_build(name, cache_dir=DEFAULT_CACHE, log=None):
    """Return (workload, base [n][d] float32, index dict)."""
    w = WORKLOADS[name]
    say = log or (lambda *_: None)
    cache = os.path.join(cache_dir, f"amp_{w.name}_{w.n}_{w.nlist}_{w.M}_{w.seed}.npz") if cache_dir else None
    t = time.perf_counter()
    if cache and os.path.exists(cache):
        z = np.load(cache, allow_pickle=False)
        base = z["base"]
        idx = {k: (z[k] if z[k].ndim else z[k].item()) for k in z.files if k != "base"}
        say(f"loaded cached base and index from {cache} in {time.perf_counter() - t:.1f}s")
        return w, base, idx
    base = make_base(w)
    say(f"generated base {base.shape} in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    idx = build_index(base, w.nlist, w.M, iters=20, seed=w.seed, integer_data=w.integer_data,
                      grid_kind=w.grid_kind, metric=w.metric)
    say(f"built IVF{w.nlist}/PQ{w.M} index in {time.perf_counter() - t:.1f}s")
    if cache:
        os.makedirs(cache_dir, exist_ok=True)
        tmp = cache + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, base=base, **idx)
        os.replace(tmp, cache)
    return w, base, idx
