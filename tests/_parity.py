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
    """Coarse distances: within 1e-3 relative of FP64 plus the FP32 expansion
    allowance fp32_coarse_tol (needed only where |D64| is far below the
    operands' magnitudes: near-zero L2 distances, near-orthogonal inner
    products).  Under L2 every distance of at least a hundredth of its
    magnitude meets the plain 1e-3 relative bar.  Returns the largest
    relative error."""
    C = np.asarray(idx["centroids"], dtype=np.float32)
    worst = 0.0
    for i, q in enumerate(Q):
        D64 = oracle.coarse_distances(q, C, idx["metric"])
        tol = 1e-3 * np.abs(D64) + fp32_coarse_tol(q, C)
        err = np.abs(gpu_coarse[i].astype(np.float64) - D64)
        assert np.all(err <= tol), (i, float(err.max()))
        if idx["metric"] == "l2":
            q64, C64 = np.asarray(q, np.float64), C.astype(np.float64)
            mag = (q64 * q64).sum() + (C64 * C64).sum(1) + 2 * np.abs(C64 @ q64)
            far = np.abs(D64) >= 1e-2 * mag
            assert np.all(err[far] <= 1e-3 * np.abs(D64[far])), i
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


def fp64_adc(idx, q, probes):
    """The full-precision oracle's FP64 ADC distance of every vector of the
    probed lists, with the magnitude its FP32 evaluation rounds against.

    Returns {id: (D64, mag)}.  mag is the sum over the vector's LUT terms of
    the absolute values that enter an FP32 evaluation of the entries and of
    their sum: L2 sum_m |r_m|^2 + |c_m|^2 + 2 |r_m . c_m|; inner product
    sum_t |q_t| (|C_pt| + |c_t|); L1 sum_t |r_t| + |c_t|."""
    metric = idx["metric"]
    C = np.asarray(idx["centroids"], np.float32)
    CB = np.asarray(idx["codebook"], np.float32)
    M = int(idx["M"])
    offs = np.asarray(idx["list_offsets"])
    codes_all = np.asarray(idx["codes"], np.int64)
    ids_all = np.asarray(idx["ids"])
    q = np.asarray(q, np.float32)
    out = {}
    for p in [int(x) for x in probes if x >= 0]:
        codes = codes_all[offs[p]:offs[p + 1]]
        if len(codes) == 0:
            continue
        rec = CB[np.arange(M)[None, :], codes].reshape(len(codes), -1).astype(np.float64)
        if metric == "ip":
            T = oracle.lut_f64(q, CB, "ip")
            add = -float(q.astype(np.float64) @ C[p].astype(np.float64))
            mag = np.abs(q.astype(np.float64)) @ (np.abs(C[p].astype(np.float64))[:, None] + np.abs(rec.T))
        else:
            r = oracle.residual_f32(q, C[p])
            T = oracle.lut_f64(r, CB, metric)
            add = 0.0
            r64 = r.astype(np.float64)
            if metric == "l2":
                dsub = CB.shape[2]
                rm = r64.reshape(M, dsub)
                cm = rec.reshape(len(codes), M, dsub)
                mag = ((rm * rm).sum(1)[None, :] + (cm * cm).sum(2) + 2 * np.abs((cm * rm[None]).sum(2))).sum(1)
            else:
                mag = (np.abs(r64)[None, :] + np.abs(rec)).sum(1)
        D = add + T[np.arange(M)[None, :], codes].sum(1)
        for v, dv, mv in zip(ids_all[offs[p]:offs[p + 1]].tolist(), D.tolist(), np.atleast_1d(mag).tolist()):
            out[v] = (dv, mv)
    return out


def fp32_adc_tol(idx, mag):
    """Bound on |D32 - D64| of one vector under the FP32 policy: each LUT
    entry is an FP32 expression of d/M + 2 terms (at most d/M + 2 roundings),
    the scan adds M entries (M - 1 roundings), the inner-product list term is
    a sum of d products, and the reported distance is rounded once more;
    with gamma_n = n 2^-24 / (1 - n 2^-24) that is at most
    gamma_(M + d/M + 4) mag for L2 and L1 and gamma_(M + d + 4) mag for the
    inner product.  The bound is taken as (that n) 2^-23 mag (twice gamma_n:
    the GPU's order of the additions is not the oracle's)."""
    M = int(idx["M"])
    dsub = int(idx["d"]) // M
    n = M + (int(idx["d"]) if idx["metric"] == "ip" else dsub) + 4
    return n * 2.0 ** -23 * mag


def compare_fp32(gpu, ref, idx, Q):
    """FP32 policy against the FP64 oracle, per returned id: every returned id
    is a distinct member of one of the query's probed lists, its reported
    distance is within fp32_adc_tol of its own FP64 ADC distance, and where
    the GPU's id at a rank differs from the oracle's, the two ids' FP64
    distances are within the sum of their bounds (a certified near-tie).
    Returns the number of rows with such swaps."""
    g_d = gpu["dist"].astype(np.float64)
    fin = np.isfinite(ref["dist"])
    assert np.array_equal(np.isfinite(g_d), fin)
    assert np.array_equal(gpu["ids"] >= 0, fin)
    probes = gpu["probes"] if "probes" in gpu else ref["probes"]
    swaps = 0
    for i, q in enumerate(Q):
        row = gpu["ids"][i][fin[i]].tolist()
        if not row:
            continue
        assert len(set(row)) == len(row), i
        D = fp64_adc(idx, q, probes[i])
        for j, v in enumerate(row):
            assert v in D, (i, j, v)
            d64, mag = D[v]
            assert abs(g_d[i, j] - d64) <= fp32_adc_tol(idx, mag), (i, j, v, g_d[i, j], d64)
        assert np.all(np.diff(g_d[i][fin[i]]) >= 0), i
        want = ref["ids"][i][fin[i]].tolist()
        if row != want:
            swaps += 1
            for a, b in zip(row, want):
                if a != b:
                    (da, ma), (db, mb) = D[a], D[b]
                    assert abs(da - db) <= fp32_adc_tol(idx, ma) + fp32_adc_tol(idx, mb), (i, a, b, da, db)
    return swaps


def bf16_bits(x):
    """bfloat16 bit patterns (uint16) of float32 values, round to nearest even
    (test input preparation: queries and base rows stored as BF16)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def bf16_widen(b):
    """float32 values of bfloat16 bit patterns (exact)."""
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)
