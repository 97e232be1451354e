"""Cluster locating with adaptive operand precision — TEST INFRASTRUCTURE.

Plain int64 / FP64 oracle of the reduced-precision CL stage: the vector space
division into dimension slices and per-slice sub-spaces (Sec. 3.1), the
sub-space features and the regression that predicts a precision per
sub-space (Sec. 3.2-3.4), and the distance module's CL pass on operands of
that precision, accumulated over the slices (Sec. 4.1 DCM / DRM; MSB-first
bit order, Sec. 4.2).  Shares no code with the HIP library.

Readings of the paper that this file fixes (where it is silent):
  * CL operands are 8-bit signed codes v = round((x - o) * 2^-ec), half to
    even, clamped to [-128, 127]; x - o is rounded once to FP32.  o is the
    FP32 midpoint of the centroids' value range (inner product: 0) and ec
    the smallest exponent with every centroid value within 127 * 2^ec of o;
  * S equal slices of consecutive dimensions; each slice's centroid codes
    are clustered into P sub-spaces (integer centres, every centroid in the
    sub-space of its nearest centre, ties to the lower index; radius = the
    ceiling of the largest member distance; count = number of members);
  * a query's features in slice s for sub-space u: d' = |vq_s - z_su|^2,
    r1 / n1 of C1 = the sub-space with the smallest d' (ties: lower index),
    r2 / n2 of u; the same fixed-point regressor as the LUT predictor
    (mitchell_log2_q8, feature_u, svr_eval) with its own model; width =
    the low width if the score is at most theta[0], else 8 bits;
  * a b-bit operand keeps the top b bits of the 8-bit two's-complement code
    (the dropped bits read as zero: floor to a multiple of 2^(8-b));
  * slice s of centroid i is computed at the width of its sub-space
    assign[i, s] for this query; D_i = sum over slices of
    sum_t (vq_t^(b) - vc_it^(b))^2 (L2) or -sum_t vq_t^(b) vc_it^(b) (inner
    product); probes = the nprobe smallest (D_i, i).
"""
from __future__ import annotations

import numpy as np

from .search import feature_u, svr_eval, select_probes

I64 = np.int64
CL_FULL = 8


def cl_params(centroids, metric):
    """Code offset o (FP32) and exponent ec of the CL operand codes."""
    C = np.asarray(centroids, dtype=np.float32)
    if metric == "ip":
        o = np.float32(0.0)
    else:
        o = np.float32((float(C.min()) + float(C.max())) / 2.0)
    A = max(float(C.max()) - float(o), float(o) - float(C.min()))
    if A <= 0:
        return o, 0
    ec = -60
    while A > 127.0 * 2.0 ** ec:
        ec += 1
    return o, ec


def cl_codes(X, o, ec):
    """8-bit signed CL codes of FP32 vectors (the reading above)."""
    diff = (np.asarray(X, dtype=np.float32) - np.float32(o)).astype(np.float32)
    v = np.rint(diff.astype(np.float64) * 2.0 ** (-int(ec)))
    return np.clip(v, -128, 127).astype(I64)


def trunc(v, b):
    """b-bit MSB-first operand of 8-bit codes: top b bits kept, the rest zero."""
    k = CL_FULL - int(b)
    return (np.asarray(v, dtype=I64) >> k) << k


def slices(d, S):
    w = d // S
    return [(s * w, (s + 1) * w) for s in range(S)]


def subspace_features(vq, clmap):
    """Per slice: d' to every sub-space centre and C1.  Returns (d2 [S, P],
    c1 [S])."""
    S, P = int(clmap["S"]), int(clmap["P"])
    Z = np.asarray(clmap["centre"], dtype=I64)  # [S, P, w]
    d2 = np.zeros((S, P), dtype=I64)
    c1 = np.zeros(S, dtype=I64)
    for s, (a, b) in enumerate(slices(len(vq), S)):
        diff = Z[s] - np.asarray(vq[a:b], dtype=I64)[None, :]
        d2[s] = (diff * diff).sum(1)
        c1[s] = np.lexsort((np.arange(P), d2[s]))[0]
    return d2, c1


def predict_cl_bits(vq, clmap, model, low):
    """PPM for CL (Sec. 3.3-3.4): width of every (slice, sub-space) for one
    query.  Returns (bits [S, P], scores [S, P] as Python ints)."""
    S, P = int(clmap["S"]), int(clmap["P"])
    r = np.asarray(clmap["radius"], dtype=I64)
    n = np.asarray(clmap["count"], dtype=I64)
    d2, c1 = subspace_features(vq, clmap)
    theta = int(np.asarray(model["theta"], dtype=I64)[0])
    bits = np.zeros((S, P), dtype=I64)
    ys = np.zeros((S, P), dtype=object)
    for s in range(S):
        for u in range(P):
            x = [int(d2[s, u]), int(r[s, c1[s]]), int(r[s, u]), int(n[s, c1[s]]), int(n[s, u])]
            y = svr_eval(feature_u(x, model), model)
            ys[s, u] = y
            bits[s, u] = int(low) if y <= theta else CL_FULL
    return bits, ys


def coarse_mixed(vq, Vc, assign, bits, S, metric):
    """DCM CL pass at per-(slice, sub-space) operand width, summed over the
    slices (Sec. 4.1).  vq [d], Vc [nlist, d] codes; assign [nlist, S];
    bits [S, P].  Exact int64 per centroid."""
    Vc = np.asarray(Vc, dtype=I64)
    assign = np.asarray(assign, dtype=I64)
    bits = np.asarray(bits, dtype=I64)
    D = np.zeros(len(Vc), dtype=I64)
    for s, (a, b) in enumerate(slices(Vc.shape[1], S)):
        k = (CL_FULL - bits[s, assign[:, s]])[:, None]  # per centroid
        qv = (np.asarray(vq[a:b], dtype=I64)[None, :] >> k) << k
        cv = (Vc[:, a:b] >> k) << k
        if metric == "ip":
            D -= (qv * cv).sum(1)
        else:
            D += ((qv - cv) ** 2).sum(1)
    return D


def cl_probes(q, index, clmap, nprobe, policy, bits=8, low=4, model=None):
    """Probes of one query under the integer CL policies.  policy "fixed":
    every partial distance at ``bits``; "adaptive": widths from the CL
    predictor (``model``), low width ``low``.  Returns (probes, D, widths
    [S, P])."""
    S, P = int(clmap["S"]), int(clmap["P"])
    vq = cl_codes(q, clmap["o"], clmap["ec"])
    Vc = cl_codes(index["centroids"], clmap["o"], clmap["ec"])
    if policy == "fixed":
        B = np.full((S, P), int(bits), dtype=I64)
    elif policy == "adaptive":
        B, _ = predict_cl_bits(vq, clmap, model, low)
    else:
        raise ValueError(policy)
    D = coarse_mixed(vq, Vc, clmap["assign"], B, S, index["metric"])
    return select_probes(D, nprobe), D, B


def low_share(B, clmap, low):
    """Fraction of one query's partial distances (centroid, slice) computed
    at the low width."""
    n = np.asarray(clmap["count"], dtype=I64)
    return float((n * (np.asarray(B) == int(low))).sum()) / float(n.sum())
