"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare them to the bar the tests state."""
from __future__ import annotations

import numpy as np

import oracle

INT64_MAX = np.iinfo(np.int64).max


def fp32_coarse_tol(q, C):
    """Error bound of the FP32 expansion |q|^2 + |c|^2 - 2 q.c against FP64:
    a few ulps of the operands' magnitudes (d-term dot products accumulate
    at most d roundings) plus the 1e-3 relative bar."""
    q = np.asarray(q, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    mag = (q * q).sum() + (C * C).sum(1) + 2 * np.abs(C @ q)
    return (len(q) + 4) * 2.0 ** -23 * mag


def check_coarse(gpu_coarse, idx, Q):
    C = np.asarray(idx["centroids"], dtype=np.float32)
    worst = 0.0
    for i, q in enumerate(Q):
        D64 = oracle.coarse_distances(q, C, idx["metric"])
        tol = 1e-3 * np.abs(D64) + fp32_coarse_tol(q, C)
        err = np.abs(gpu_coarse[i].astype(np.float64) - D64)
        assert np.all(err <= tol), (i, float(err.max()))
        worst = max(worst, float((err / np.maximum(np.abs(D64), 1e-30)).max()))
    return worst


def certify_probes(gpu_probes, idx, Q, nprobe):
    """Probe sets must equal the oracle's, except where the FP64 distances of
    the differing lists are within the FP32 expansion error of each other
    (certified near-ties).  Returns the number of certified near-ties."""
    C = np.asarray(idx["centroids"], dtype=np.float32)
    ties = 0
    npq = np.broadcast_to(np.asarray(nprobe), (len(Q),))
    for i, q in enumerate(Q):
        D64 = oracle.coarse_distances(q, C, idx["metric"])
        want = oracle.select_probes(D64, int(npq[i]))
        got = gpu_probes[i][: int(npq[i])]
        if np.array_equal(got, want):
            continue
        tol = fp32_coarse_tol(q, C)
        # every position where the two orders differ must be a near-tie
        for a, b in zip(got.tolist(), want.tolist()):
            if a != b:
                assert abs(D64[a] - D64[b]) <= tol[a] + tol[b], (i, a, b, D64[a], D64[b])
        ties += 1
    return ties


def compare_integer(gpu, ref):
    """Bit-exact ids, integer distances and float distances."""
    assert np.array_equal(gpu["ids"], ref["ids"]), _first_diff(gpu["ids"], ref["ids"])
    assert np.array_equal(gpu["qdist"], ref["qdist"]), _first_diff(gpu["qdist"], ref["qdist"])
    assert np.array_equal(gpu["dist"].view(np.uint32), ref["dist"].view(np.uint32))


def _first_diff(a, b):
    bad = np.argwhere(a != b)
    if len(bad) == 0:
        return "equal"
    i, j = bad[0]
    return f"first difference at query {i} rank {j}: {a[i, j]} vs {b[i, j]}; row gpu {a[i]} ref {b[i]}"


def compare_fp32(gpu, ref, M):
    """FP32 policy: distances within the FP32 summation bound of the FP64
    ones, ids equal except where the FP64 distances are that close."""
    g_d = gpu["dist"].astype(np.float64)
    r_d = ref["dist"].astype(np.float64)
    fin = np.isfinite(r_d)
    assert np.array_equal(np.isfinite(g_d), fin)
    scale = np.where(fin, np.abs(r_d), 0).max(1, keepdims=True) + 1e-30
    # FP32 sums of M entries, each formed as |r|^2 + |c|^2 - 2 r.c: a few
    # ulps of the row's distance scale; 1e-4 relative stays well inside the
    # 1e-3 bar
    tol = 1e-4 * scale
    diff = np.zeros_like(g_d)
    diff[fin] = g_d[fin] - r_d[fin]
    assert np.all(np.abs(diff) <= tol)
    mism = gpu["ids"] != ref["ids"]
    for i, j in np.argwhere(mism):
        # a swapped id must sit among distances within the bound
        assert abs(g_d[i, j] - r_d[i, j]) <= tol[i, 0], (i, j)
    return int(mism.any(1).sum())


def bf16_bits(x):
    """bfloat16 bit patterns (uint16) of float32 values, round to nearest even
    (test input preparation: queries and base rows stored as BF16)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def bf16_widen(b):
    """float32 values of bfloat16 bit patterns (exact)."""
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)
