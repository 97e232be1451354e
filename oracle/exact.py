"""Brute-force exact k-nearest neighbours in FP64 and recall (test infrastructure)."""
from __future__ import annotations

import numpy as np


def exact_knn(base, queries, k, metric="l2"):
    """Exact top-k ids by (distance, id) over the raw vectors, FP64.

    ``metric`` "l2": squared Euclidean distance; "l1": sum of absolute
    differences; "ip": negative inner product.
    """
    B = np.asarray(base, dtype=np.float64)
    n = len(B)
    out = np.full((len(queries), k), -1, dtype=np.int64)
    for i, q in enumerate(np.asarray(queries, dtype=np.float64)):
        if metric in ("l2", "l1"):
            D = np.empty(n)
            for s in range(0, n, 1 << 16):
                diff = B[s:s + (1 << 16)] - q
                D[s:s + (1 << 16)] = (diff * diff).sum(1) if metric == "l2" else np.abs(diff).sum(1)
        else:
            D = -(B @ q)
        kk = min(k, n)
        kth = np.partition(D, kk - 1)[kk - 1]
        cand = np.flatnonzero(D <= kth)
        order = np.lexsort((cand, D[cand]))[:kk]
        out[i, :kk] = cand[order]
    return out


def recall_at(found, truth, r=None):
    """k-recall@r: |found[:, :r] ∩ truth| / |truth| averaged over queries."""
    found = np.asarray(found)
    truth = np.asarray(truth)
    r = r or found.shape[1]
    hits = [len(set(f[:r].tolist()) & set(t.tolist())) for f, t in zip(found, truth)]
    return float(np.mean(hits)) / truth.shape[1]


def recall_1_at(found, truth, r=None):
    """1-recall@r: fraction of queries whose exact nearest neighbour is among
    the first r returned ids."""
    found = np.asarray(found)
    truth = np.asarray(truth)
    r = r or found.shape[1]
    return float(np.mean([t[0] in set(f[:r].tolist()) for f, t in zip(found, truth)]))
