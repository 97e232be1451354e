"""Error statements of the integer LUT path against FP64 — TEST
INFRASTRUCTURE (a report computed by the oracle, not part of the search).

For each workload shape (scaled so that the oracle finishes in seconds) and
each LUT width b, on a sample of (query, probed list) pairs:
  * grid error of LC: |T_int * h^2 - T64| / max_j |T64[m][j]| per row
    (max and RMS), T64 the FP64 LUT of the FP32 residual and codebook;
  * ADC distance error: |D~ * h^2 - D64| over the pair's vectors, relative
    to the mean |D64| of the pair (percentiles; inner-product distances cross
    zero, so the pair's scale rather than each distance), D64 the FP64 ADC
    distance, D~ the quantised estimate;
  * the bound M * 2^(s-1) on |D~ - D_int| (Sec. 4.1 quantiser reading) is
    checked on every vector;
  * recall@10 of the FIXED-b search and of the FP32 policy against exact kNN.
The integer path of the GPU equals the oracle bit for bit, so these figures
are the GPU's.  Run: python -m oracle.error_report
"""
from __future__ import annotations

import numpy as np

from .exact import exact_knn, recall_at
from .search import (coarse_distances, grid, index_grid, lut_f64, lut_int, quantize_lut, residual_f32,
                     search, select_probes)

F64 = np.float64


def lut_errors(idx, Q, nprobe, widths=(4, 8, 12, 16)):
    M = int(idx["M"])
    e = int(idx["grid_e"])
    h2 = 2.0 ** (2 * e)
    inv = 2.0 ** (-e)
    metric, kind = idx["metric"], idx["grid_kind"]
    cbi, ci = index_grid(idx)
    C = np.asarray(idx["centroids"], np.float32)
    CB = np.asarray(idx["codebook"], np.float32)
    offs, codes = idx["list_offsets"], np.asarray(idx["codes"], np.int64)
    row_err = []
    d_err = {b: [] for b in widths}
    bound_ok = True
    for q in Q:
        P = select_probes(coarse_distances(q, C, metric), nprobe)
        for p in P:
            if metric == "l2":
                r = residual_f32(q, C[p])
                T64 = lut_f64(r, CB, "l2")
                Ti = lut_int(grid(r.astype(F64) * inv, kind), cbi, "l2")
                extra_i, extra64 = 0, 0.0
            else:
                qi = grid(q.astype(F64) * inv, kind)
                T64 = lut_f64(q, CB, "ip")
                Ti = lut_int(qi, cbi, "ip")
                extra_i = -int((qi * ci[p]).sum())
                extra64 = -float(q.astype(F64) @ C[p].astype(F64))
            rowmax = np.abs(T64).max(1, keepdims=True) + 1e-300
            row_err.append((np.abs(Ti * h2 - T64) / rowmax).ravel())
            c = codes[offs[p]:offs[p + 1]]
            if len(c) == 0:
                continue
            sel = (np.arange(M)[None, :], c)
            D64 = extra64 + T64[sel].sum(1)
            Dint = extra_i + Ti[sel].sum(1)
            for b in widths:
                Qt, s, base = quantize_lut(Ti, b)
                Dq = extra_i + base + (Qt[sel].sum(1) << s)
                if s and np.abs(Dq - Dint).max() > M * (1 << (s - 1)):
                    bound_ok = False
                d_err[b].append(np.abs(Dq * h2 - D64) / max(float(np.abs(D64).mean()), 1e-300))
    row_err = np.concatenate(row_err)
    out = dict(lut_max=float(row_err.max()), lut_rms=float(np.sqrt((row_err ** 2).mean())), bound_ok=bound_ok)
    for b in widths:
        v = np.concatenate(d_err[b])
        out[f"adc_b{b}"] = [float(np.percentile(v, 50)), float(np.percentile(v, 99)), float(v.max())]
    return out


def recalls(idx, base, Q, k, nprobe, widths=(4, 8, 12, 16)):
    truth = exact_knn(base, Q, k, idx["metric"])
    out = {"fp32": recall_at(search(idx, Q, k, nprobe, policy="fp32")["ids"], truth)}
    for b in widths:
        out[f"b{b}"] = recall_at(search(idx, Q, k, nprobe, policy="fixed", bits=b)["ids"], truth)
    return out


def main():
    from amp_data import build_index
    from amp_data.synth import WORKLOADS, make_base, make_queries

    shapes = [
        ("tiny (20k x 32, IVF64/PQ8, U9 grid)", WORKLOADS["tiny"], 8, 40),
        ("mid shape (60k x 128 integer, IVF128/PQ16, h = 1)", WORKLOADS["mid"].scaled(n=60_000, nlist=128),
         16, 20),
        ("skewed shape (100k x 96 Zipf, IVF256/PQ24)", WORKLOADS["skewed"].scaled(n=100_000, nlist=256), 32, 20),
        ("highdim shape (20k x 960 aniso, IVF64/PQ120, e4m3 grid)", WORKLOADS["highdim"].scaled(n=20_000, nlist=64),
         8, 8),
        ("serving shape (50k x 768 unit, inner product, IVF128/PQ96)",
         WORKLOADS["serving"].scaled(n=50_000, nlist=128), 16, 8),
    ]
    print("| workload | LC grid error max / RMS (of row max) | ADC rel. error p50 / p99 / max at b = 4, 8, 12, 16 "
          "| bound M 2^(s-1) | recall@10 FP32 / b4 / b8 / b12 / b16 |")
    print("|---|---|---|---|---|")
    for name, w, nprobe, nq in shapes:
        base = make_base(w)
        idx = build_index(base, w.nlist, w.M, iters=8, seed=w.seed, integer_data=w.integer_data,
                          grid_kind=w.grid_kind, metric=w.metric)
        Q = make_queries(w, nq)
        le = lut_errors(idx, Q[: min(nq, 8)], min(nprobe, 8))
        rc = recalls(idx, base, Q, 10, nprobe)
        adc = "; ".join("/".join(f"{x:.1e}" for x in le[f"adc_b{b}"]) for b in (4, 8, 12, 16))
        print(f"| {name} | {le['lut_max']:.1e} / {le['lut_rms']:.1e} | {adc} | "
              f"{'holds' if le['bound_ok'] else 'VIOLATED'} | {rc['fp32']:.3f} / {rc['b4']:.3f} / {rc['b8']:.3f} / "
              f"{rc['b12']:.3f} / {rc['b16']:.3f} |", flush=True)


if __name__ == "__main__":
    main()
