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


def replicate(idx, copies):
    """An index whose every list holds `copies` copies of the original list
    (ids of copy c offset by c * N): the same clusters and codes at `copies`
    times the size, for measurements on a working set larger than the GPU's
    last-level cache.  Duplicate vectors tie in distance; results are not
    meant for recall."""
    offs = np.asarray(idx["list_offsets"], np.int64)
    ids = np.asarray(idx["ids"], np.int64)
    codes = np.asarray(idx["codes"])
    n = len(ids)
    sizes = np.diff(offs)
    new_offs = np.concatenate([[0], np.cumsum(sizes * copies)]).astype(np.int64)
    new_ids = np.empty(n * copies, np.int64)
    new_codes = np.empty((n * copies, codes.shape[1]), codes.dtype)
    for p in range(len(sizes)):
        a, b = offs[p], offs[p + 1]
        o = new_offs[p]
        for c in range(copies):
            new_ids[o + c * (b - a): o + (c + 1) * (b - a)] = ids[a:b] + c * n
            new_codes[o + c * (b - a): o + (c + 1) * (b - a)] = codes[a:b]
    out = dict(idx)
    out.update(list_offsets=new_offs, ids=new_ids, codes=new_codes,
               list_sizes=(sizes * copies).astype(np.int32))
    return out
