"""FP64 / int64 oracle of the batched IVF-PQ search with cluster-adaptive LUT
precision — TEST INFRASTRUCTURE (see the package docstring).

Stages, in the paper's order (Sec. 2.1, Fig. 1):
  CL  cluster locating: distance from the query to every centroid, keep the
      nprobe nearest;
  RC  residual between the query and each probed centroid;
  LC  look-up table of the residual's distance to every codeword of every
      subspace (complete, no pruning: Sec. 3.3, Sec. 6);
  PPM precision of each probed cluster predicted from {d', r1, r2, n1, n2}
      by an RBF support-vector regressor evaluated with a table (Sec. 3.3-3.4,
      Sec. 4.1);
  DC  distance of each vector of the cluster = sum of its codes' LUT entries;
      b-bit LUT values are widened to a common width before the sum (Sec. 4.1,
      DRM);
  TS  top-k by (distance, id) over all probed clusters (Sec. 4.1, TSM).

Readings of the paper that this file fixes (where it is silent):
  * "precision" of a probed cluster = the width b in {4, 8, 12, 16} of its
    quantised LUT entries; LUT operands live on an integer grid of step
    h = 2**e (9-bit signed integers, or integers exactly representable in
    FP8 e4m3), so the integer LUT is exact;
  * quantisation per (query, probed cluster): subtract each subspace's
    minimum, one power-of-two shift s shared by the whole LUT, rounding half
    up; the distance estimate is base + (sum << s);
  * d' = squared norm of the grid residual; r = radius in grid units;
    n = list size; C1 = the probed cluster with the smallest d' (ties: lower
    list id);  features enter the regressor through a fixed-point
    base-2 logarithm (Mitchell's approximation) and an integer affine map;
  * ties: probes by (distance, list id); results by (distance, id).

Everything here is plain loops over queries and probes with numpy on whole
arrays; no blocking, fusion or reordering beyond the definitions.
"""
from __future__ import annotations

import numpy as np

F64 = np.float64
I64 = np.int64
KSUB = 256
BITS_ALL = (4, 8, 12, 16)


# --------------------------------------------------------------------- CL
def coarse_distances(q, centroids, metric="l2"):
    """CL (Sec. 2.1): distance from one query to every centroid, FP64.

    L2: sum_t (q_t - c_t)^2.  L1 (the distance module's second mode,
    Sec. 4.1): sum_t |q_t - c_t|.  IP: -sum_t q_t c_t.
    """
    q = np.asarray(q, dtype=F64)
    C = np.asarray(centroids, dtype=F64)
    if metric == "l2":
        diff = C - q[None, :]
        return (diff * diff).sum(1)
    if metric == "l1":
        return np.abs(C - q[None, :]).sum(1)
    return -(C @ q)


def select_probes(D, nprobe):
    """CL selection (Sec. 2.1, TSM in Sec. 4.1): the nprobe smallest by
    (distance, list id)."""
    D = np.asarray(D)
    order = np.lexsort((np.arange(len(D)), D))
    return order[:nprobe].astype(np.int64)


# --------------------------------------------------------------------- RC
def residual_f32(q, c):
    """RC (Sec. 2.1): r = q - c, rounded once to FP32.

    The difference of two FP32 numbers is formed in FP64 and rounded to FP32;
    with 53 >= 2*24 + 2 significand bits the double rounding is innocuous, so
    this equals the correctly rounded FP32 subtraction.
    """
    return (np.asarray(q, dtype=F64) - np.asarray(c, dtype=F64)).astype(np.float32)


def e4m3_round_int(v):
    """Round integers to the nearest value representable in OCP FP8 E4M3
    (round half to even on the 3-bit mantissa; saturate to +-448)."""
    v = np.asarray(v, dtype=I64)
    a = np.abs(v)
    out = a.copy()
    big = a >= 16
    if np.any(big):
        ab = a[big]
        E = np.floor(np.log2(ab.astype(F64))).astype(I64)
        # guard against log2 rounding at exact powers of two
        E = np.where((1 << (E + 1)) <= ab, E + 1, E)
        E = np.where((1 << E) > ab, E - 1, E)
        step = I64(1) << (E - 3)
        qt, rem = np.divmod(ab, step)
        half = step >> 1
        up = (rem > half) | ((rem == half) & (qt % 2 == 1))
        out[big] = (qt + up) * step
    out = np.minimum(out, 448)
    return np.sign(v) * out


def grid(x_scaled, kind="u9"):
    """Map values already divided by the grid step onto the operand grid.

    "u9": round half to even to an integer, saturate to [-255, 255];
    "e4m3": round half to even to an integer, then to the nearest E4M3 value
    (half to even, saturating at 448).
    """
    v = np.rint(np.asarray(x_scaled, dtype=F64)).astype(I64)
    if kind == "u9":
        return np.clip(v, -255, 255)
    return e4m3_round_int(v)


def index_grid(index):
    """Codebook (and, for IP, centroids) on the operand grid of the index."""
    e = int(index["grid_e"])
    kind = index["grid_kind"]
    inv = 2.0 ** (-e)
    cbi = grid(np.asarray(index["codebook"], dtype=F64) * inv, kind)
    ci = grid(np.asarray(index["centroids"], dtype=F64) * inv, kind)
    return cbi, ci


# --------------------------------------------------------------------- LC
def lut_int(ri, cbi, metric="l2"):
    """LC (Sec. 2.1) on the integer grid, exact int64.

    L2: T[m][j] = sum_{t in m} (ri_t - cbi[m][j][t])^2.
    L1: T[m][j] = sum_{t in m} |ri_t - cbi[m][j][t]|.
    IP: T[m][j] = -sum_{t in m} qi_t * cbi[m][j][t].
    """
    M, ksub, dsub = cbi.shape
    r = np.asarray(ri, dtype=I64).reshape(M, 1, dsub)
    if metric == "l2":
        diff = r - cbi
        return (diff * diff).sum(2)
    if metric == "l1":
        return np.abs(r - cbi).sum(2)
    return -(r * cbi).sum(2)


def lut_f64(r, codebook, metric="l2"):
    """LC for the full-precision policy: FP64 arithmetic on the FP32 operands."""
    CB = np.asarray(codebook, dtype=F64)
    M, ksub, dsub = CB.shape
    rr = np.asarray(r, dtype=F64).reshape(M, 1, dsub)
    if metric == "l2":
        diff = rr - CB
        return (diff * diff).sum(2)
    if metric == "l1":
        return np.abs(rr - CB).sum(2)
    return -(rr * CB).sum(2)


def quantize_lut(T, b, granularity="pair"):
    """b-bit LUT of one (query, probed cluster) pair (Sec. 4.1 DRM: b-bit
    entries widened to a common width before accumulation).

    lo_m = min_j T[m][j];  R_m = max_j (T[m][j] - lo_m);  hf(s) = 2^(s-1) (0 if s = 0);
    granularity "pair" (one width for every subspace, Sec. 1 cluster level):
      s = smallest s >= 0 with (max_m R_m + hf(s)) >> s <= 2^b - 1;
    granularity "subspace" (a width per (pair, subspace), Sec. 5.3: the
    pair's lane budget M (2^b - 1) shared by its subspaces in proportion to
    their ranges, subspace m carrying about log2(R_m >> s) bits):
      s = smallest s >= 0 with (sum_m R_m + M hf(s)) >> s <= M (2^b - 1);
    Q = (T - lo_m + hf(s)) >> s;  base = sum_m lo_m.
    Returns (Q, s, base).
    """
    T = np.asarray(T, dtype=I64)
    lo = T.min(1)
    Rm = (T - lo[:, None]).max(1)
    if granularity == "pair":
        R, n = int(Rm.max()), 1
    elif granularity == "subspace":
        R, n = int(Rm.sum()), len(Rm)
    else:
        raise ValueError(granularity)
    top = n * ((1 << b) - 1)
    s = 0
    while ((R + n * (1 << (s - 1) if s else 0)) >> s) > top:
        s += 1
    hf = (1 << (s - 1)) if s else 0
    Q = (T - lo[:, None] + hf) >> s
    return Q, s, int(lo.sum())


# --------------------------------------------------------------------- PPM
def mitchell_log2_q8(x):
    """Fixed-point log2(x + 1) with 8 fraction bits, by Mitchell's piecewise
    linear approximation (J. N. Mitchell, 1962): for y = x + 1 with leading
    bit k, log2 y ~ k + (y / 2^k - 1)."""
    y = np.asarray(x, dtype=I64) + 1
    out = np.zeros(y.shape, dtype=I64)
    flat_y = y.reshape(-1)
    flat_o = out.reshape(-1)
    for i, yy in enumerate(flat_y.tolist()):
        k = int(yy).bit_length() - 1
        flat_o[i] = 256 * k + ((int(yy) << 8) >> k) - 256
    return out


def feature_u(x5, model):
    """Integer affine map of the log-features onto the 10-bit grid 0..1023."""
    L = mitchell_log2_q8(np.asarray(x5, dtype=I64))
    lo = np.asarray(model["feat_lo"], dtype=I64)
    mul = np.asarray(model["feat_mul"], dtype=I64)
    return np.clip(((L - lo) * mul) >> 16, 0, 1023)


def svr_eval(u5, model):
    """RBF support-vector regression with the kernel read from a table
    (Sec. 3.4): y = beta0 + sum_i beta_i * table[min(1023, (g * ||u - s_i||^2) >> 32)].
    All integer; y is in Q40."""
    u = np.asarray(u5, dtype=I64)
    sv = np.asarray(model["sv"], dtype=I64)
    dist2 = ((sv - u[None, :]) ** 2).sum(1)
    idx = np.minimum((dist2 * int(model["g_mul"])) >> 32, len(model["table"]) - 1)
    K = np.asarray(model["table"], dtype=I64)[idx]
    beta = np.asarray(model["beta"], dtype=I64)
    return int(model["beta0"]) + int((beta * K).sum())


def bits_from_score(y, model, allowed=BITS_ALL, margin_q40=0):
    """Smallest allowed width whose threshold admits y (+ margin); if none,
    the largest allowed width.  Thresholds exist for 4, 8 and 12 bits."""
    allowed = sorted(allowed)
    theta = list(np.asarray(model["theta"], dtype=I64).tolist()) + [None]
    for b in allowed:
        t = theta[b // 4 - 1]
        if t is None or y + margin_q40 <= t:
            return b
    return allowed[-1]


def predict_pair_bits(dq2, probes, radq, sizes, model, allowed=BITS_ALL, margin_q40=0):
    """PPM (Sec. 3.3, Sec. 4.1) for all probed clusters of one query.

    Features of pair (q, p): d' = dq2[p], r1 = radq[C1], r2 = radq[p],
    n1 = |C1|, n2 = |p|, where C1 is the probed cluster with the smallest d'
    (ties: lower list id).  Returns (bits per probe, score per probe).
    """
    dq2 = np.asarray(dq2, dtype=I64)
    probes = np.asarray(probes, dtype=I64)
    c1 = probes[np.lexsort((probes, dq2))[0]]
    bits, ys = [], []
    for i, p in enumerate(probes.tolist()):
        x = [int(dq2[i]), int(radq[c1]), int(radq[p]), int(sizes[c1]), int(sizes[p])]
        y = svr_eval(feature_u(x, model), model)
        ys.append(y)
        bits.append(bits_from_score(y, model, allowed, margin_q40))
    return np.asarray(bits, dtype=I64), np.asarray(ys, dtype=object)


# --------------------------------------------------------------------- DC + TS
def dc_ts(index, P, tables, k):
    """DC and TS (Sec. 2.1; Sec. 4.1 DRM, TSM) of one query on the integer
    path, given each probed cluster's quantised LUT: for every vector v of
    probed list P[j], S_v = sum_m Q_j[m][code_v,m] and D_v = base_j + (S_v << s_j);
    then the k smallest (D, id).  ``tables``: one (Q [M][256], s, base) per
    probe.  Returns (ids [k], D [k]) padded with (-1, INT64_MAX)."""
    M = int(index["M"])
    offs = np.asarray(index["list_offsets"], dtype=I64)
    ids_all = np.asarray(index["ids"], dtype=I64)
    codes_all = np.asarray(index["codes"], dtype=I64)
    cand_d, cand_id = [], []
    for p, (Qt, s, base) in zip(np.asarray(P).tolist(), tables):
        codes = codes_all[offs[p]:offs[p + 1]]
        S = np.asarray(Qt, dtype=I64)[np.arange(M)[None, :], codes].sum(1)
        cand_d.append(int(base) + (S << int(s)))
        cand_id.append(ids_all[offs[p]:offs[p + 1]])
    Dall = np.concatenate(cand_d) if cand_d else np.zeros(0, I64)
    Iall = np.concatenate(cand_id) if cand_id else np.zeros(0, I64)
    order = np.lexsort((Iall, Dall))[:k]
    out_i = np.full(k, -1, dtype=I64)
    out_d = np.full(k, np.iinfo(I64).max, dtype=I64)
    out_i[:len(order)] = Iall[order]
    out_d[:len(order)] = Dall[order]
    return out_i, out_d


# --------------------------------------------------------------------- search
def _per_query(v, nq):
    v = np.asarray(v)
    return np.full(nq, int(v)) if v.ndim == 0 else v.astype(np.int64)


def search(index, queries, k, nprobe, policy="fixed", bits=16, allowed=BITS_ALL,
           model=None, explicit_bits=None, margin_q40=0, probes=None, cl=None, granularity="pair"):
    """Full search of a query batch.

    policy: "fp32" (full-precision LUT), "fixed" (every pair at ``bits``),
    "adaptive" (predictor, ``model``), "explicit" (``explicit_bits`` [nq, npmax]
    by probe rank).  ``probes`` [nq, npmax] (-1 padded) overrides CL's
    selection (used to continue from another implementation's probe set when
    the two differ only by a certified near-tie).  ``cl`` selects the
    integer CL on 8-bit codes (oracle.cl): a dict with "map" (the index's
    sub-space map), "policy" ("fixed" at "bits", or "adaptive" with "model"
    and low width "low").  ``granularity``: the quantiser's ("pair" or
    "subspace", see quantize_lut).

    Returns a dict: ids [nq, kmax] int64, qdist [nq, kmax] int64 (-1 for fp32),
    dist [nq, kmax] float32, probes, bits, shift, base [nq, npmax].
    """
    Q = np.asarray(queries, dtype=np.float32)
    nq, d = Q.shape
    M = int(index["M"])
    metric = index["metric"]
    e = int(index["grid_e"])
    inv = 2.0 ** (-e)
    # distance unit of an integer estimate: h^2 (L2, IP: products of two grid
    # values), h (L1: sums of grid values)
    h2 = 2.0 ** (e if metric == "l1" else 2 * e)
    kq = _per_query(k, nq)
    npq = _per_query(nprobe, nq)
    kmax, npmax = int(kq.max()), int(npq.max())
    C = np.asarray(index["centroids"], dtype=np.float32)
    CB = np.asarray(index["codebook"], dtype=np.float32)
    offs = np.asarray(index["list_offsets"], dtype=I64)
    ids_all = np.asarray(index["ids"], dtype=I64)
    codes_all = np.asarray(index["codes"], dtype=I64)
    sizes = np.asarray(index["list_sizes"], dtype=I64)
    radq = np.asarray(index["radq"], dtype=I64)
    cbi, ci = index_grid(index)
    out_ids = np.full((nq, kmax), -1, dtype=I64)
    out_q = np.full((nq, kmax), np.iinfo(I64).max, dtype=I64)
    out_d = np.full((nq, kmax), np.inf, dtype=np.float32)
    out_p = np.full((nq, npmax), -1, dtype=I64)
    out_b = np.zeros((nq, npmax), dtype=I64)
    out_s = np.zeros((nq, npmax), dtype=I64)
    out_base = np.zeros((nq, npmax), dtype=I64)
    for i in range(nq):
        q = Q[i]
        # CL
        if probes is None and cl is not None:
            from .cl import cl_probes
            P, _, _ = cl_probes(q, index, cl["map"], int(npq[i]), cl["policy"], cl.get("bits", 8),
                                cl.get("low", 4), cl.get("model"))
        elif probes is None:
            P = select_probes(coarse_distances(q, C, metric), int(npq[i]))
        else:
            P = np.asarray(probes[i], dtype=I64)
            P = P[P >= 0]
        out_p[i, :len(P)] = P
        cand_d, cand_id = [], []
        if policy == "fp32":
            for p in P.tolist():
                if metric in ("l2", "l1"):
                    T = lut_f64(residual_f32(q, C[p]), CB, metric)
                    add = 0.0
                else:
                    T = lut_f64(q, CB, metric)
                    add = float(-(q.astype(F64) @ C[p].astype(F64)))
                codes = codes_all[offs[p]:offs[p + 1]]
                Dv = add + T[np.arange(M)[None, :], codes].sum(1)
                cand_d.append(Dv)
                cand_id.append(ids_all[offs[p]:offs[p + 1]])
            Dall = np.concatenate(cand_d) if cand_d else np.zeros(0)
            Iall = np.concatenate(cand_id) if cand_id else np.zeros(0, I64)
            order = np.lexsort((Iall, Dall))[: kq[i]]
            out_ids[i, :len(order)] = Iall[order]
            out_q[i, :] = -1
            out_d[i, :len(order)] = Dall[order].astype(np.float32)
            continue
        # RC on the grid (L2 and L1: the residual; IP: the query)
        if metric in ("l2", "l1"):
            RI = [grid(residual_f32(q, C[p]).astype(F64) * inv, index["grid_kind"])
                  for p in P.tolist()]
        else:
            qi = grid(q.astype(F64) * inv, index["grid_kind"])
            RI = [qi - ci[p] for p in P.tolist()]
        dq2 = np.asarray([int((r * r).sum()) for r in RI], dtype=I64)
        # PPM
        if policy == "fixed":
            B = np.full(len(P), bits, dtype=I64)
        elif policy == "explicit":
            B = np.asarray(explicit_bits[i][:len(P)], dtype=I64)
        elif policy == "adaptive":
            B, _ = predict_pair_bits(dq2, P, radq, sizes, model, allowed, margin_q40)
        else:
            raise ValueError(policy)
        out_b[i, :len(P)] = B
        if metric == "ip":
            T_query = lut_int(qi, cbi, "ip")
        tables = []
        for j, p in enumerate(P.tolist()):
            # LC
            if metric in ("l2", "l1"):
                T = lut_int(RI[j], cbi, metric)
                extra = 0
            else:
                T = T_query
                extra = -int((qi * ci[p]).sum())
            Qt, s, base = quantize_lut(T, int(B[j]), granularity)
            base += extra
            out_s[i, j] = s
            out_base[i, j] = base
            tables.append((Qt, s, base))
        # DC + TS
        oi, od = dc_ts(index, P, tables, int(kq[i]))
        kk = int(kq[i])
        out_ids[i, :kk] = oi
        out_q[i, :kk] = od
        fin = oi >= 0
        out_d[i, :kk][fin] = od[fin].astype(np.float32) * np.float32(h2)
    return dict(ids=out_ids, qdist=out_q, dist=out_d, probes=out_p, bits=out_b,
                shift=out_s, base=out_base)
