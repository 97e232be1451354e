"""IVF-PQ index construction for the synthetic workloads (Sec. 2.1).

The corpus is split into ``nlist`` clusters by k-means; every vector's
residual to its centroid is split into ``M`` contiguous sub-vectors, each
encoded by the index of the nearest of 256 codewords of a codebook shared by
all clusters; the codes of each cluster are stored contiguously.  Per cluster
the builder also records its size and radius (Sec. 3.3 uses both as features
of the precision predictor).

Conventions fixed here (the paper leaves them open):
  * k-means: initial centroids are distinct points of a seeded sample, at most
    ``256 * k`` training points, a fixed number of Lloyd iterations, ties to
    the lowest centroid index, an empty cluster takes the training point that
    is farthest from its current centroid;
  * integer data: centroids and codewords are rounded to integers after
    training and every vector is re-assigned, so that all distances are exact
    integers (the paper's 8-bit operands, Sec. 5.3);
  * members of a list are stored in increasing id order;
  * ``grid_e``: the operand grid step of the LUT build is h = 2**grid_e, the
    smallest power of two with max(|codeword entry|, |residual entry|) / h
    (inner product: also |centroid entry| and |vector entry|) within the
    grid's largest magnitude (255 for the 9-bit integer grid, 448 for the e4m3
    grid); integer data uses h = 1;
  * ``radq``: the radius max ||x - c||_2 in grid units, rounded to nearest.
"""
from __future__ import annotations

import numpy as np

KSUB = 256
GRID_MAX = {"u9": 255.0, "e4m3": 448.0}


def _rng(seed, purpose):
    return np.random.Generator(np.random.PCG64([seed, 77, purpose]))


def _sqnorms(X):
    X = X.astype(np.float32, copy=False)
    return np.einsum("ij,ij->i", X, X, dtype=np.float32)


def assign(X, C, chunk=1 << 16):
    """Nearest centroid (squared L2, ties -> lowest index) and its distance."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    C = np.ascontiguousarray(C, dtype=np.float32)
    cn = _sqnorms(C)
    a = np.empty(len(X), dtype=np.int64)
    dist = np.empty(len(X), dtype=np.float32)
    for s in range(0, len(X), chunk):
        x = X[s:s + chunk]
        D = cn[None, :] - 2.0 * (x @ C.T)
        D += _sqnorms(x)[:, None]
        a[s:s + chunk] = np.argmin(D, axis=1)
        dist[s:s + chunk] = D[np.arange(len(x)), a[s:s + chunk]]
    return a, dist


def kmeans(X, k, iters, seed, max_train_per_centroid=256):
    X = np.ascontiguousarray(X, dtype=np.float32)
    n = len(X)
    r = _rng(seed, 0)
    ntrain = min(n, max_train_per_centroid * k)
    sample = X if ntrain == n else X[np.sort(r.choice(n, ntrain, replace=False))]
    # distinct initial centroids from a seeded permutation
    perm = r.permutation(len(sample))
    picked, seen = [], set()
    for i in perm:
        key = sample[i].tobytes()
        if key in seen:
            continue
        seen.add(key)
        picked.append(i)
        if len(picked) == k:
            break
    if len(picked) < k:
        # fewer distinct points than centroids: repeat them (the duplicates
        # are never chosen by the lowest-index tie rule)
        picked = [picked[i % len(picked)] for i in range(k)]
    C = sample[np.asarray(picked)].astype(np.float64)
    for _ in range(iters):
        a, dist = assign(sample, C)
        counts = np.bincount(a, minlength=k)
        order = np.argsort(a, kind="stable")
        starts = np.searchsorted(a[order], np.arange(k))
        nonempty = counts > 0
        sums = np.zeros((k, X.shape[1]), dtype=np.float64)
        red = np.add.reduceat(sample[order].astype(np.float64), starts[nonempty], axis=0)
        sums[nonempty] = red
        newC = C.copy()
        newC[nonempty] = sums[nonempty] / counts[nonempty, None]
        empty = np.flatnonzero(~nonempty)
        if len(empty):
            far = np.argsort(-dist.astype(np.float64), kind="stable")
            for e_i, c in enumerate(empty):
                newC[c] = sample[far[e_i % len(far)]]
        C = newC
    return C.astype(np.float32)


def build_index(base, nlist, M, iters=20, seed=0, integer_data=False,
                grid_kind="u9", metric="l2", ids=None):
    """Build the IVF-PQ index arrays for ``base`` [n, d] float32."""
    base = np.ascontiguousarray(base, dtype=np.float32)
    n, d = base.shape
    if d % M:
        raise ValueError("d must be a multiple of M")
    dsub = d // M
    C = kmeans(base, nlist, iters, seed)
    if integer_data:
        C = np.rint(C)
    a, _ = assign(base, C)
    resid = base - C[a]
    # residual product quantiser: one 256-word codebook per subspace, shared
    # by all clusters
    r = _rng(seed, 1)
    ntrain = min(n, 256 * KSUB)
    samp = resid if ntrain == n else resid[np.sort(r.choice(n, ntrain, replace=False))]
    CB = np.empty((M, KSUB, dsub), dtype=np.float32)
    for m in range(M):
        sub = np.ascontiguousarray(samp[:, m * dsub:(m + 1) * dsub])
        CB[m] = kmeans(sub, KSUB, iters, seed + 1000 + m)
    if integer_data:
        CB = np.rint(CB)
    codes = np.empty((n, M), dtype=np.uint8)
    for m in range(M):
        codes[:, m] = assign(resid[:, m * dsub:(m + 1) * dsub], CB[m])[0]
    if ids is None:
        ids = np.arange(n, dtype=np.int64)
    ids = np.asarray(ids, dtype=np.int64)
    order = np.lexsort((ids, a))
    sizes = np.bincount(a, minlength=nlist).astype(np.int64)
    offsets = np.zeros(nlist + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    # per-list radius (FP64) and the grid step
    rad = np.zeros(nlist, dtype=np.float64)
    rn = np.sqrt(np.einsum("ij,ij->i", resid.astype(np.float64), resid.astype(np.float64)))
    np.maximum.at(rad, a, rn)
    if integer_data:
        e = 0
    else:
        A = max(float(np.abs(CB).max()), float(np.abs(resid).max()))
        if metric == "ip":
            # inner product puts queries and centroids on the grid
            A = max(A, float(np.abs(C).max()), float(np.abs(base).max()))
        e = int(np.ceil(np.log2(A / GRID_MAX[grid_kind])))
    h = 2.0 ** e
    return dict(
        d=d, M=M, dsub=dsub, nlist=nlist, ksub=KSUB, metric=metric,
        grid_kind=grid_kind, grid_e=e,
        centroids=C.astype(np.float32), codebook=CB.astype(np.float32),
        list_offsets=offsets, ids=ids[order], codes=codes[order],
        list_sizes=sizes.astype(np.int32), radius=rad,
        radq=np.rint(rad / h).astype(np.int32),
    )


def lossless_index(seed, nlist, M, dsub, per_list, cb_range=6, c_range=40):
    """Hand-built index whose base vectors are exactly centroid + codewords.

    Centroids and codewords are small integers, so every vector of list p is
    reproduced exactly by its code; with all lists probed, the ADC distance
    then equals the exact distance.  Returns (index arrays, base [n, d]) where
    base rows follow the ids 0..n-1.
    """
    r = _rng(seed, 2)
    d = M * dsub
    C = r.integers(-c_range, c_range + 1, size=(nlist, d)).astype(np.float32)
    CB = r.integers(-cb_range, cb_range + 1, size=(M, KSUB, dsub)).astype(np.float32)
    sizes = np.asarray(per_list, dtype=np.int64)
    if sizes.shape == ():
        sizes = np.full(nlist, int(sizes))
    n = int(sizes.sum())
    offsets = np.zeros(nlist + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    codes = r.integers(0, KSUB, size=(n, M)).astype(np.uint8)
    lists = np.repeat(np.arange(nlist), sizes)
    recon = CB[np.arange(M)[None, :], codes.astype(np.int64)].reshape(n, d)
    base_sorted = C[lists] + recon
    # ids: a seeded permutation, increasing inside each list
    ids = np.empty(n, dtype=np.int64)
    pid = r.permutation(n)
    for p in range(nlist):
        ids[offsets[p]:offsets[p + 1]] = np.sort(pid[offsets[p]:offsets[p + 1]])
    base = np.empty_like(base_sorted)
    base[ids] = base_sorted
    rn = np.sqrt(((base_sorted - C[lists]).astype(np.float64) ** 2).sum(1))
    rad = np.zeros(nlist)
    np.maximum.at(rad, lists, rn)
    idx = dict(
        d=d, M=M, dsub=dsub, nlist=nlist, ksub=KSUB, metric="l2", grid_kind="u9",
        grid_e=0, centroids=C, codebook=CB, list_offsets=offsets, ids=ids,
        codes=codes, list_sizes=sizes.astype(np.int32), radius=rad,
        radq=np.rint(rad).astype(np.int32),
    )
    return idx, base
