"""Throughput benchmark of the adaptive-precision IVF-PQ search on one MI355X.

Default run (the JSON line the driver records): the largest single-GPU
workload, the serving corpus (5M x 768 unit-normalised BF16 rows from a
2048-component mixture, inner product, IVF2048 / PQ96x256, index built on
the device).  A step is one search of a batch of 4096 BF16 queries with
per-query k in {10, 50, 100} and nprobe in {16, 64, 256} (the serving mix,
sizes resident on the device, one captured HIP graph replayed): coarse
distances, probe selection, precision prediction, work queue, LUT build +
quantisation + scan, top-k merge.  Queries, sizes and the index are resident
in HBM before the timed region.  `value` is the adaptive policy's QPS; the
full-precision (FP32 LUT) policy is timed the same way beside it, recall@10
of both is taken over every query of the batch against exact FP64 search,
and one Poisson arrival rate through the serving loop gives p50 / p99.  The
mid-size workload (1M x 128 integer data, IVF1024 / PQ16, 10 000 queries,
nprobe 32, k 10) is measured the same way as a secondary field.  A
per-policy table goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KIND_TEXT = {"uint8": "integer-valued Gaussian mixture", "iso": "isotropic Gaussian mixture",
             "zipf": "Zipf(1.1)-weighted Gaussian mixture", "aniso": "anisotropic Gaussian mixture",
             "vmf": "unit-normalised mixture"}
HBM_PEAK_GBS = 8000.0
FP32_MFMA_TFLOPS = 157.3
BF16_MFMA_TFLOPS = 2500.0
# 32-bit VALU lane operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_scan_mid_traffic.json")
TRAFFIC_FILE_C5 = os.path.join(ROOT, "profiles", "k_scan_serving_traffic.json")
STREAM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_scan_stream_traffic.json")


def _kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "scan_kernels.h", "device_common.h", "amp_internal.h"):
        with open(os.path.join(ROOT, "paper_2606_07156_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per launch of the phase-2 scan from the committed counter
    summary, if it was taken on the current kernel source (else None)."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    return t.get("bytes_per_launch") if t.get("kernel_hash") == _kernel_hash() else None


def recall_1(ids, truth):
    """1-recall@10: share of queries whose exact nearest neighbour is among
    the 10 returned ids."""
    ids, truth = np.asarray(ids)[:, :10], np.asarray(truth)
    return float(np.mean([truth[i, 0] in set(ids[i].tolist()) for i in range(len(ids))]))


def recall_10(ids, truth):
    """10-recall@10: mean share of the exact top 10 among the 10 returned."""
    ids, truth = np.asarray(ids)[:, :10], np.asarray(truth)[:, :10]
    return float(np.mean([len(set(ids[i].tolist()) & set(truth[i].tolist())) / 10.0 for i in range(len(ids))]))


def exact_knn_device(base, Q, k, metric, chunk=1 << 18):
    """Exact top-k ids by (distance, id) in FP64 on the device (ground truth
    for recall on corpora too large for the host brute force)."""
    import torch
    dev = torch.device("cuda:0")
    q = torch.from_numpy(np.asarray(Q, np.float64)).to(dev)
    qn = (q * q).sum(1, keepdim=True)
    best = torch.full((len(Q), k), float("inf"), dtype=torch.float64, device=dev)
    bid = torch.zeros((len(Q), k), dtype=torch.int64, device=dev)
    for s in range(0, len(base), chunk):
        x = torch.from_numpy(np.asarray(base[s:s + chunk], np.float64)).to(dev)
        D = -(q @ x.T) if metric == "ip" else qn + (x * x).sum(1)[None, :] - 2.0 * (q @ x.T)
        ids = torch.arange(s, s + len(x), device=dev).expand(len(Q), -1)
        D2, I2 = torch.cat([best, D], 1), torch.cat([bid, ids], 1)
        # order by (distance, id): ids break ties
        o = torch.argsort(I2, dim=1, stable=True)
        D2, I2 = torch.gather(D2, 1, o), torch.gather(I2, 1, o)
        o = torch.argsort(D2, dim=1, stable=True)[:, :k]
        best, bid = torch.gather(D2, 1, o), torch.gather(I2, 1, o)
    return bid.cpu().numpy()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cpu_worker(args):
    import oracle
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)  # one thread per worker process
    except ImportError:
        pass
    idx, Q, k, nprobe, kw = args
    t = time.perf_counter()
    oracle.search(idx, Q, k, nprobe, **kw)
    return time.perf_counter() - t


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(idx, Q, k, nprobe, kw, budget_s=20.0, max_procs=16):
    """Time the oracle on a bounded sample of the same queries, one
    single-threaded worker process per host core (at most `max_procs`: the
    host's CPU share for one GPU)."""
    cores = min(os.cpu_count() or 1, max_procs)
    kk = np.broadcast_to(np.asarray(k), (len(Q),))
    nn = np.broadcast_to(np.asarray(nprobe), (len(Q),))
    t0 = time.perf_counter()
    _cpu_worker((idx, Q[:2], kk[:2], nn[:2], kw))
    per_q = max((time.perf_counter() - t0) / 2, 1e-4)
    n = int(min(len(Q), max(cores, budget_s * cores / per_q)))
    n = max(cores, (n // cores) * cores)
    chunks = [(idx, Q[:n][i::cores], kk[:n][i::cores], nn[:n][i::cores], kw) for i in range(cores)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_cpu_worker, chunks)
    wall = time.perf_counter() - t0
    return dict(value=round(n / wall, 2), unit="queries/s", cores=cores, kind="oracle",
                cpu=cpu_model(), host_cpus=os.cpu_count(),
                sample=f"first {n} of {len(Q)} queries of the timed batch (interleaved over {cores} "
                       f"single-threaded processes), {wall:.1f} s wall")


def serving_base_on_device(w, dev, chunk=1 << 19):
    """The serving corpus at full size, drawn on the device: the workload's
    mixture (means, weights and sigma of amp_data.synth), component labels
    from numpy's seeded generator, Gaussian noise from torch's seeded device
    generator, rows normalised and rounded to bfloat16 (nearest-even).
    Returns the BF16 bit patterns [n][d] uint16 on the host."""
    import torch
    from amp_data.synth import _mixture_params
    means, weights, sigma = _mixture_params(w)
    comp = np.random.Generator(np.random.PCG64([w.seed, 9001])).choice(w.n_comp, size=w.n, p=weights)
    g = torch.Generator(device=dev)
    g.manual_seed(w.seed * 1000 + 17)
    mu = torch.from_numpy(means.astype(np.float32)).to(dev)
    sg = torch.from_numpy(sigma.astype(np.float32)).to(dev)
    ct = torch.from_numpy(comp.astype(np.int64)).to(dev)
    out = np.empty((w.n, w.d), np.uint16)
    for s in range(0, w.n, chunk):
        e = min(w.n, s + chunk)
        x = mu[ct[s:e]] + torch.randn((e - s, w.d), generator=g, device=dev) * sg
        x = x / x.norm(dim=1, keepdim=True)
        out[s:e] = x.to(torch.bfloat16).view(torch.int16).cpu().numpy().view(np.uint16)
    return out


def serving(args):
    """Serving regime: single-query requests of mixed k and nprobe arriving
    as a Poisson process at each rate lambda, continuously batched by the
    library's server; latency from the scheduled arrival to the results in
    host memory."""
    import torch

    import paper_2606_07156_amd as amp
    from amp_data.synth import WORKLOADS, make_queries

    w = WORKLOADS["serving"]
    if args.serve_n:
        w = w.scaled(n=args.serve_n)
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    b16 = serving_base_on_device(w, dev)
    torch.cuda.synchronize()
    log(f"[serve] generated {b16.shape} bf16 corpus in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    h = amp.amp_index_build(b16, w.nlist, w.M, iters=20, seed=w.seed, metric="ip", grid_kind=w.grid_kind)
    arr = amp.amp_index_get_arrays(h)
    sizes = np.diff(arr["list_offsets"])
    log(f"[serve] built IVF{w.nlist}/PQ{w.M} on the device in {time.perf_counter() - t:.1f}s; list sizes "
        f"min/mean/max {sizes.min()}/{sizes.mean():.0f}/{sizes.max()}, grid_e {arr['grid_e']}")
    del arr
    t = time.perf_counter()
    TQ = make_queries(w, args.train_queries, train=True)
    rep = amp.amp_index_train_predictor(h, TQ, 10, 64, gamma=args.gamma, epsilon=args.epsilon, C_=args.svr_c,
                                        n_samples=1280)
    log(f"[serve] trained predictor in {time.perf_counter() - t:.1f}s: {rep}")
    R = args.requests
    Q = make_queries(w, R)  # bf16-representable rows
    Qb = np.ascontiguousarray((Q.view(np.uint32) >> 16).astype(np.uint16))
    r = np.random.Generator(np.random.PCG64([w.seed, 9002]))
    ks = np.array([10, 50, 100], np.int32)[r.integers(0, 3, R)]
    nps = np.array([16, 64, 256], np.int32)[r.integers(0, 3, R)]
    ids = np.zeros((R, 100), np.int64)
    dist = np.zeros((R, 100), np.float32)
    qaddr = Qb.ctypes.data + np.arange(R, dtype=np.int64) * Qb.strides[0]
    iaddr = ids.ctypes.data + np.arange(R, dtype=np.int64) * ids.strides[0]
    daddr = dist.ctypes.data + np.arange(R, dtype=np.int64) * dist.strides[0]

    # recall@10 of the batched search at each nprobe: adaptive and FP32 vs
    # exact inner-product search (FP64 on the device over the BF16 corpus)
    nr = min(args.recall_queries, R)
    recall = {}
    if nr:
        xb = torch.from_numpy(b16.view(np.int16)).to(dev).view(torch.bfloat16)
        qq = torch.from_numpy(Q[:nr].astype(np.float64)).to(dev)
        best = torch.full((nr, 10), -float("inf"), dtype=torch.float64, device=dev)
        bid = torch.zeros((nr, 10), dtype=torch.int64, device=dev)
        for s in range(0, w.n, 1 << 20):
            sc = qq @ xb[s:s + (1 << 20)].to(torch.float64).T
            v, i = torch.topk(torch.cat([best, sc], 1), 10, dim=1)
            bid = torch.gather(torch.cat([bid, torch.arange(s, s + sc.shape[1], device=dev).expand(nr, -1)], 1), 1, i)
            best = v
        truth = bid.cpu().numpy()
        del xb
        for npb in (16, 64, 256):
            for pol in ("adaptive", "fp32"):
                g = amp.amp_search(h, Qb[:nr], 10, npb, policy=pol, want_bits=True)
                rec = float(np.mean([len(set(g["ids"][i]) & set(truth[i])) / 10 for i in range(nr)]))
                recall[f"{pol}_nprobe{npb}"] = round(rec, 4)
                if pol == "adaptive":
                    bits = g["bits"][:, :npb].ravel()
                    recall[f"bits_nprobe{npb}"] = {int(b): round(float((bits == b).mean()), 3) for b in np.unique(bits)}
        log(f"[serve] 10-recall@10 over {nr} queries: {recall}")

    def make_server(policy):
        return amp.amp_server_create(h, max_batch=args.serve_batch, max_pending=65536, max_k=100, max_nprobe=256,
                                     q_dtype="bf16", policy=policy)

    def run(srv, lam, n):
        """open loop: request i is due at its Poisson arrival time (lam <= 0:
        all due at once, the closed-loop capacity)"""
        gaps = r.exponential(1.0 / lam, n) if lam > 0 else np.zeros(n)
        due = (np.cumsum(gaps) * 1e9).astype(np.int64)
        rejected = 0
        lag = 0
        t0 = time.monotonic_ns() + 2_000_000
        for i in range(n):
            a = t0 + int(due[i])
            now = time.monotonic_ns()
            while now < a:
                if a - now > 200_000:
                    time.sleep((a - now - 100_000) * 1e-9)
                now = time.monotonic_ns()
            lag = max(lag, now - a)
            j = i % R
            if srv.submit_raw(int(qaddr[j]), int(ks[j]), int(nps[j]), int(iaddr[j]), int(daddr[j]), 0, a) != 0:
                rejected += 1
        amp.amp_server_flush(srv)
        st = amp.amp_server_stats(srv, reset=True)
        st["max_submit_lag_ms"] = lag / 1e6
        return st

    rows = []
    for pol in args.serve_policies.split(","):
        srv = make_server(pol)
        run(srv, 0, min(R, 4096))  # warm-up
        cap = run(srv, 0, R)
        log(f"[serve] {pol}: closed-loop capacity {cap['qps']:.0f} QPS, mean batch {cap['mean_batch']:.0f}, "
            f"p50 {cap['p50_ms']:.2f} ms p99 {cap['p99_ms']:.2f} ms")
        rows.append(dict(policy=pol, lam="capacity", qps=round(cap["qps"], 1), p50_ms=round(cap["p50_ms"], 3),
                         p99_ms=round(cap["p99_ms"], 3), mean_batch=round(cap["mean_batch"], 1)))
        for lam in [float(x) for x in args.lambdas.split(",")] if pol == args.serve_policies.split(",")[0] else []:
            n = min(R, max(1000, int(lam * args.serve_seconds)))
            st = run(srv, lam, n)
            log(f"[serve] {pol} lambda {lam:.0f}: {n} requests, achieved {st['qps']:.0f} QPS, p50 "
                f"{st['p50_ms']:.3f} ms, p99 {st['p99_ms']:.3f} ms, max {st['max_ms']:.2f} ms, mean batch "
                f"{st['mean_batch']:.1f}, rejected {st['rejected']}, submit lag max {st['max_submit_lag_ms']:.2f} ms")
            rows.append(dict(policy=pol, lam=lam, requests=n, qps=round(st["qps"], 1), p50_ms=round(st["p50_ms"], 3),
                             p99_ms=round(st["p99_ms"], 3), max_ms=round(st["max_ms"], 3),
                             mean_batch=round(st["mean_batch"], 1), rejected=st["rejected"],
                             submit_lag_max_ms=round(st["max_submit_lag_ms"], 3)))
        srv.close()
    head = [x for x in rows if x["lam"] != "capacity"]
    line = {
        "metric": "p99 latency at Poisson arrival rate (serving)",
        "value": head[-1]["p99_ms"] if head else None,
        "unit": "ms",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n}x{w.d} bf16 unit-normalised mixture ({w.n_comp} components), "
                               f"inner product, IVF{w.nlist}/PQ{w.M}x256, k in {{10,50,100}}, "
                               f"nprobe in {{16,64,256}}, BF16 queries, one query per request",
                   "server": {"max_batch": args.serve_batch, "max_pending": 65536},
                   "recall_10_at_10": recall},
        "serving": rows,
    }
    print(json.dumps(line), flush=True)


def sweep(args):
    """Batched uneven work: the skewed workload (10M x 96, Zipf(1.1) mixture
    weights, IVF4096 / PQ24) searched in batches of B queries with per-query
    nprobe uniform in [8, 128], k 10; adaptive (BF16 LC) and FP32 policies,
    each with its schedule autotuned per batch size."""
    import torch

    import paper_2606_07156_amd as amp
    from amp_data.synth import WORKLOADS, draw_nprobe, make_base, make_queries

    w = WORKLOADS["skewed"]
    if args.serve_n:
        w = w.scaled(n=args.serve_n)
    t = time.perf_counter()
    base = make_base(w)
    log(f"[sweep] generated base {base.shape} in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    h = amp.amp_index_build(base, w.nlist, w.M, iters=20, seed=w.seed)
    arr = amp.amp_index_get_arrays(h)
    sizes = np.diff(arr["list_offsets"])
    log(f"[sweep] built IVF{w.nlist}/PQ{w.M} on the device in {time.perf_counter() - t:.1f}s; list sizes "
        f"min/median/mean/max {sizes.min()}/{int(np.median(sizes))}/{sizes.mean():.0f}/{sizes.max()}")
    TQ = make_queries(w, args.train_queries, train=True)
    rep = amp.amp_index_train_predictor(h, TQ, 10, 64, gamma=args.gamma, epsilon=args.epsilon, C_=args.svr_c,
                                        n_samples=1280)
    log(f"[sweep] trained predictor: {rep}")
    bmax = max(int(b) for b in args.batches.split(","))
    Q = make_queries(w, max(bmax, w.nq))
    NP = draw_nprobe(w, len(Q))
    t = time.perf_counter()
    truth = exact_knn_device(base, Q[:bmax], 10, w.metric)
    log(f"[sweep] exact kNN of {bmax} queries in {time.perf_counter() - t:.1f}s")
    del base
    dev = torch.device("cuda:0")
    qd = torch.from_numpy(Q).to(dev)
    npd = torch.from_numpy(NP.astype(np.int32)).to(dev)
    kd = torch.full((len(Q),), 10, dtype=torch.int32, device=dev)
    stream = torch.cuda.Stream()
    rows = []
    for B in [int(b) for b in args.batches.split(",")]:
        for pol in ("adaptive", "fp32"):
            kw = dict(policy=pol)
            e = amp.amp_index_autotune(h, Q[:B], 10, NP[:B], repeats=3, **kw)
            out = dict(ids=torch.empty((B, 10), dtype=torch.int64, device=dev),
                       dist=torch.empty((B, 10), dtype=torch.float32, device=dev))
            szs = dict(k=kd[:B], nprobe=npd[:B], kmax=10, npmax=int(NP.max()))
            reps = max(3, min(200, int(2000 / max(B, 1)) + 3))
            for i in range(2):
                amp.amp_search(h, qd[:B], out=out, stream=stream, graph=True, **szs, **kw)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for i in range(reps):
                amp.amp_search(h, qd[:B], out=out, stream=stream, graph=True, **szs, **kw)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            ids = out["ids"].cpu().numpy()
            r1, r10 = recall_1(ids, truth[:B]), recall_10(ids, truth[:B])
            rows.append(dict(batch=B, policy=pol, ms=round(ms, 4), qps=round(B / ms * 1e3, 1),
                             recall_1_at_10=round(r1, 4), recall_10_at_10=round(r10, 4),
                             schedule={kk: e[kk] for kk in ("chunk", "chunk1", "narrow", "lut_dtype", "queue")},
                             tuned_ms=round(e["ms"], 4), automatic_ms=round(e["ms_default"], 4)))
            log(f"[sweep] B={B:5d} {pol:8s} {ms:8.3f} ms/batch {B / ms * 1e3:11.0f} QPS  1-recall@10 {r1:.4f} "
                f"10-recall@10 {r10:.4f}  schedule {rows[-1]['schedule']} (tuned {e['ms']:.3f} ms vs automatic "
                f"{e['ms_default']:.3f} ms)")
    line = {"metric": "QPS per batch size (batched uneven work)", "unit": "queries/s", "n_gpus": 1,
            "higher_is_better": True, "data": "synthetic",
            "config": {"workload": f"{w.name}: {w.n}x{w.d} Zipf(1.1) mixture, IVF{w.nlist}/PQ{w.M}x256, "
                                   f"nprobe uniform in [{w.nprobe_lo},{w.nprobe}], k 10",
                       "list_sizes": [int(sizes.min()), int(np.median(sizes)), int(sizes.max())]},
            "sweep": rows}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="",
                    help="one named workload with constant k / nprobe instead of the default run")
    ap.add_argument("--nq", type=int, default=0)
    ap.add_argument("--policies", default="adaptive,fp32")
    ap.add_argument("--train-queries", type=int, default=256)
    ap.add_argument("--gamma", type=float, default=10.0)
    ap.add_argument("--epsilon", type=float, default=0.1)
    ap.add_argument("--svr-c", type=float, default=1.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--granularity", type=int, default=1,
                    help="1: also measure per-(pair, subspace) LUT widths (retrained predictor)")
    ap.add_argument("--cl-slices", type=int, default=16, help="mid workload: CL dimension slices (0: no CL run)")
    ap.add_argument("--cl-subspaces", type=int, default=64, help="mid workload: CL sub-spaces per slice")
    ap.add_argument("--cl-epsilon", type=float, default=0.1, help="epsilon of the CL predictor's SVR")
    ap.add_argument("--recall", type=int, default=1,
                    help="0: skip the exact ground truth of the headline (profiling runs); recall is then null")
    ap.add_argument("--recall-queries", type=int, default=200, help="--serving: queries checked for recall")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--serve-rate", type=float, default=10000.0,
                    help="Poisson arrival rate of the default run's serving measurement (0: skip)")
    ap.add_argument("--secondary", type=int, default=1, help="1: measure the mid-size workload after the headline")
    ap.add_argument("--cache-dir", default="/tmp/amp_bench_cache")
    ap.add_argument("--replicate", type=int, default=0,
                    help="R > 1: every list R times larger (working set beyond the last-level cache; "
                         "use with a small --nq for the streaming regime)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: autotune each policy's search schedule for the batch before timing it")
    ap.add_argument("--gpu-build", action="store_true",
                    help="build the index on the device (amp_index_build) instead of the cached numpy build")
    ap.add_argument("--allowed", default="4,8,12,16", help="widths the adaptive policy may choose")
    ap.add_argument("--schedule", default="",
                    help="chunk,chunk1,narrow,lut_dtype[,queue]: use this search schedule instead of autotuning")
    ap.add_argument("--sweep", action="store_true",
                    help="batch-size sweep on the skewed workload (uneven nprobe, Zipf list sizes)")
    ap.add_argument("--batches", default="1,16,256,1024,4096")
    ap.add_argument("--serving", action="store_true",
                    help="serving regime: Poisson arrivals of single-query requests on the serving workload")
    ap.add_argument("--lambdas", default="2000,5000,10000,20000,50000")
    ap.add_argument("--requests", type=int, default=100_000, help="request pool of the serving regime")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="arrival window per rate")
    ap.add_argument("--serve-batch", type=int, default=1024)
    ap.add_argument("--serve-policies", default="adaptive,fp32")
    ap.add_argument("--serve-n", type=int, default=0, help="corpus size override (testing)")
    args = ap.parse_args()
    if args.sweep:
        if args.gpus != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        return sweep(args)
    if args.serving:
        if args.gpus != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        return serving(args)
    if args.calibrate_copy_mb:
        import torch
        n = args.calibrate_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(1, args.steps)):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.calibrate_copy_mb} MiB x {max(1, args.steps)}")
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU path is a design "
              "note and is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.workload:
        return single(args)
    return headline(args)


# ---------------------------------------------------------------- measurement
def policy_list(names, allowed):
    pols = []
    for p in names.split(","):
        if p == "fp32":
            pols.append(("fp32", dict(policy="fp32")))
        elif p == "adaptive":
            pols.append(("adaptive", dict(policy="adaptive", allowed=allowed)))
        elif p.startswith("fixed"):
            pols.append((p, dict(policy="fixed", bits=int(p[5:]))))
    return pols


def measure(h, w, Q, kq, npq, pols, args, truth, tag, qdev=None, q_dtype=None):
    """Time every policy on one batch: W warm-up searches, then K searches
    enqueued back to back on one created stream (graph replays; per-query
    sizes, if any, resident on the device) between HIP events on that
    stream.  Then K synchronised searches with per-stage events and the
    phase-2 work counters, and one search of the whole batch for recall@10
    against `truth` (exact FP64 ids of every query)."""
    import torch

    import paper_2606_07156_amd as amp
    dev = torch.device("cuda:0")
    nq = len(Q)
    per_query = np.ndim(kq) > 0
    kmax = int(np.max(kq))
    npmax = int(np.max(npq))
    qd = qdev if qdev is not None else torch.from_numpy(Q).to(dev)
    if per_query:
        kd = torch.from_numpy(np.ascontiguousarray(kq, np.int32)).to(dev)
        npd = torch.from_numpy(np.ascontiguousarray(npq, np.int32)).to(dev)
        sizes = dict(k=kd, nprobe=npd, kmax=kmax, npmax=npmax)
    else:
        sizes = dict(k=int(kq), nprobe=int(npq))
    out = dict(ids=torch.empty((nq, kmax), dtype=torch.int64, device=dev),
               dist=torch.empty((nq, kmax), dtype=torch.float32, device=dev),
               qdist=torch.empty((nq, kmax), dtype=torch.int64, device=dev),
               status=torch.zeros(1, dtype=torch.int32, device=dev))
    stream = torch.cuda.Stream()  # a created stream of default priority (graph capture needs one)
    list_sizes = None
    results = {}
    for name, kw in pols:
        if q_dtype:
            kw = dict(kw, q_dtype=q_dtype)
        sched = "automatic"
        if args.autotune:
            tk = {kk: v for kk, v in kw.items() if kk not in ("q_dtype", "cl_policy", "cl_bits")}
            e = amp.amp_index_autotune(h, Q, kq, npq, repeats=3, **tk)
            sched = {kk: e[kk] for kk in ("chunk", "chunk1", "narrow", "lut_dtype", "queue", "ms", "ms_default")}
            log(f"[{tag}] {name}: autotuned schedule {sched}")
        for _ in range(args.warmup):
            amp.amp_search(h, qd, out=out, stream=stream, graph=True, **sizes, **kw)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            amp.amp_search(h, qd, out=out, stream=stream, graph=True, **sizes, **kw)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        status = int(out["status"].item())
        stages, works = [], []
        for _ in range(args.steps):
            o = amp.amp_search(h, qd, out=out, stream=stream, stage_ms=True, work=True, **sizes, **kw)
            stages.append(o["stage_ms"])
            works.append(o["work"])
        cl_adaptive = kw.get("cl_policy") == "adaptive"
        g = amp.amp_search(h, Q, kq, npq, want_probes=True, want_bits=True, want_cl_bits=cl_adaptive, **kw)
        cl_share = None
        if cl_adaptive:
            # share of the (query, centroid, slice) partial distances at the low width
            cm = amp.amp_index_get_cl_map(h)
            low = kw.get("cl_bits") or 4
            cl_share = float(((g["cl_bits"] == low) * cm["count"][None]).sum()) / (nq * cm["count"].sum())
        ids10 = g["ids"][:, :10]
        rec1 = recall_1(ids10, truth[:, :10]) if truth is not None else None
        rec10 = recall_10(ids10, truth[:, :10]) if truth is not None else None
        pr = g["probes"]
        bits = g["bits"][pr >= 0]
        hist = {int(b): round(float((bits == b).mean()), 4) for b in np.unique(bits)}
        if list_sizes is None:
            list_sizes = args.idx_sizes
        probed_bytes = float(list_sizes[pr[pr >= 0]].sum()) * w.M
        wk = {kk: float(np.mean([x[kk] for x in works])) for kk in works[0]}
        st = {s_: float(np.mean([x[s_] for x in stages])) for s_ in stages[0]}
        lat = [x["total"] for x in stages]
        results[name] = dict(qps=nq / (ms / 1e3), ms=ms, recall1=rec1, recall10=rec10, stages=st, status=status,
                             cl_low_share=cl_share,
                             probed_bytes=probed_bytes, scan_bytes=wk["scan_bytes"], unit_bytes=wk["unit_bytes"],
                             live_pairs=wk["live_pairs"],
                             dead_pairs=wk["dead_pairs"], bits=hist, schedule=sched,
                             n_pairs=int((pr >= 0).sum()),
                             p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)))
        log(f"[{tag}] {name:8s} {ms:8.3f} ms/step {nq / ms * 1e3:12.0f} QPS  1-recall@10 {rec1}  "
            f"10-recall@10 {rec10}  status {status}  bits {hist}  "
            + " ".join(f"{s_}={v:.3f}" for s_, v in st.items()))
    return results


def roofline_of(r, w, nq, traffic_file):
    """Roofline of the dominant kernel of the headline search: the phase-2
    scan (LUT of its pairs, then the packed-lane scan of the live pairs'
    codes).  The per-unit figure is what one work unit of the kernel reads:
    its list chunk's codes once, however many (query, list) pairs it serves
    (up to eight per LUT word), plus its LUT sources (inner product: the
    live pairs' quantised tables); achieved = those bytes summed over the
    units the launch scans (the search's own work counter) over the
    kernel's average duration, against the HBM peak.  The per-pair code
    bytes (each live pair reading its list once) exceed what the kernel
    moves by the pairs a unit shares and are context only, as are the
    probed bytes and the pairs the bound drops before any scan."""
    scan_ms = r["stages"]["scan2"]
    gbs = r["unit_bytes"] / (scan_ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(traffic_file),
            "kernel": "k_scan_mix (phase-2 scan, every lane class in one launch)",
            "kernel_ms": round(scan_ms, 4), "bytes_per_launch": round(r["unit_bytes"]),
            "context": {"live_pairs": round(r["live_pairs"]), "skipped_pairs": round(r["dead_pairs"]),
                        "pair_code_bytes": round(r["scan_bytes"]),
                        "pair_code_gbs": round(r["scan_bytes"] / (scan_ms / 1e3) / 1e9, 1),
                        "probed_code_bytes": round(r["probed_bytes"])}}


def mfma_of(r, w, nq):
    st = r["stages"]
    cl_flops = 2.0 * nq * w.nlist * w.d
    lc_flops = r["n_pairs"] * 2.0 * 256 * w.d
    cl_tf = cl_flops / (st["cl"] / 1e3) / 1e12
    lc_tf = lc_flops / ((st["base"] + st["scan1"] + st["scan2"]) / 1e3) / 1e12
    return {"cl": {"flop_per_search": cl_flops, "tflops": round(cl_tf, 2), "peak": FP32_MFMA_TFLOPS,
                   "frac": round(cl_tf / FP32_MFMA_TFLOPS, 4)},
            "lc": {"flop_per_search": lc_flops, "tflops_over_scan": round(lc_tf, 2), "peak": BF16_MFMA_TFLOPS,
                   "frac": round(lc_tf / BF16_MFMA_TFLOPS, 4)}}


def summary(results):
    rnd = lambda v: round(v, 4) if v is not None else None
    return {n: {"qps": round(x["qps"], 1), "ms": round(x["ms"], 4), "1_recall_at_10": rnd(x["recall1"]),
                **({"cl_low_share": rnd(x["cl_low_share"])} if x.get("cl_low_share") is not None else {}),
                "10_recall_at_10": rnd(x["recall10"]), "scan2_ms": round(x["stages"]["scan2"], 4),
                "stages_ms": {kk: round(v, 4) for kk, v in x["stages"].items()}, "bits_share": x["bits"],
                "device_status": x["status"]}
            for n, x in results.items()}


def serve_once(h, Qb, ks, nps, lam, seconds, policy, max_batch):
    """Open-loop Poisson arrivals at rate lam through the serving loop;
    latency from the scheduled arrival to the results in host memory."""
    import paper_2606_07156_amd as amp
    R = len(Qb)
    ids = np.zeros((R, 100), np.int64)
    dist = np.zeros((R, 100), np.float32)
    qaddr = Qb.ctypes.data + np.arange(R, dtype=np.int64) * Qb.strides[0]
    iaddr = ids.ctypes.data + np.arange(R, dtype=np.int64) * ids.strides[0]
    daddr = dist.ctypes.data + np.arange(R, dtype=np.int64) * dist.strides[0]
    srv = amp.amp_server_create(h, max_batch=max_batch, max_pending=65536, max_k=100, max_nprobe=256,
                                q_dtype="bf16", policy=policy)
    r = np.random.Generator(np.random.PCG64([7, 9003]))

    def run(lam_, n):
        gaps = r.exponential(1.0 / lam_, n) if lam_ > 0 else np.zeros(n)
        due = (np.cumsum(gaps) * 1e9).astype(np.int64)
        t0 = time.monotonic_ns() + 2_000_000
        lag = 0
        for i in range(n):
            a = t0 + int(due[i])
            now = time.monotonic_ns()
            while now < a:
                if a - now > 200_000:
                    time.sleep((a - now - 100_000) * 1e-9)
                now = time.monotonic_ns()
            lag = max(lag, now - a)
            j = i % R
            srv.submit_raw(int(qaddr[j]), int(ks[j]), int(nps[j]), int(iaddr[j]), int(daddr[j]), 0, a)
        amp.amp_server_flush(srv)
        st = amp.amp_server_stats(srv, reset=True)
        st["max_submit_lag_ms"] = lag / 1e6
        return st

    run(0, min(R, 2048))  # warm-up: every size bucket's graph captured
    n = max(1000, int(lam * seconds))
    st = run(lam, n)
    srv.close()
    return dict(policy=policy, arrival_qps=lam, requests=n, achieved_qps=round(st["qps"], 1),
                p50_ms=round(st["p50_ms"], 3), p99_ms=round(st["p99_ms"], 3), max_ms=round(st["max_ms"], 3),
                mean_batch=round(st["mean_batch"], 1), rejected=st["rejected"], failed=st["failed"],
                submit_lag_max_ms=round(st["max_submit_lag_ms"], 3))


def exact_ip_bf16(b16, Q, k, dev, chunk=1 << 20):
    """Exact inner-product top-k (FP64 on the device) over a BF16 corpus,
    ties to the lower id."""
    import torch
    xb = torch.from_numpy(b16.view(np.int16)).to(dev).view(torch.bfloat16)
    out = []
    for q0 in range(0, len(Q), 1024):
        qq = torch.from_numpy(np.asarray(Q[q0:q0 + 1024], np.float64)).to(dev)
        nr = len(qq)
        best = torch.full((nr, k), -float("inf"), dtype=torch.float64, device=dev)
        bid = torch.zeros((nr, k), dtype=torch.int64, device=dev)
        for s in range(0, len(b16), chunk):
            sc = qq @ xb[s:s + chunk].to(torch.float64).T
            ids = torch.arange(s, s + sc.shape[1], device=dev).expand(nr, -1)
            S2, I2 = torch.cat([best, sc], 1), torch.cat([bid, ids], 1)
            o = torch.argsort(I2, dim=1, stable=True)
            S2, I2 = torch.gather(S2, 1, o), torch.gather(I2, 1, o)
            o = torch.argsort(-S2, dim=1, stable=True)[:, :k]
            best, bid = torch.gather(S2, 1, o), torch.gather(I2, 1, o)
        out.append(bid.cpu().numpy())
    del xb
    return np.concatenate(out)


def apply_schedule(amp, h, args, allowed, nq):
    """--schedule chunk,chunk1,narrow,lut_dtype[,queue]: that search schedule
    for every measured policy at this batch size, instead of autotuning."""
    if not args.schedule:
        return
    f = [int(x) for x in args.schedule.split(",")]
    ents = []
    for name, kw in policy_list(args.policies, allowed):
        ents.append(dict(policy_kind=amp.POLICIES[kw["policy"]], nq_log2=int(np.ceil(np.log2(nq))),
                         chunk=f[0], chunk1=f[1], narrow=f[2], lut_dtype=f[3], queue=f[4] if len(f) > 4 else 0))
    amp.amp_index_set_tuning(h, ents)
    args.autotune = 0


def headline(args):
    """The default run: the serving workload at full size (5M x 768 BF16,
    inner product) as an offline batch with the serving mix of k and nprobe,
    adaptive vs FP32 at recall@10 over the whole batch, one Poisson arrival
    rate through the serving loop, then the mid-size workload as a secondary
    field."""
    import torch

    import paper_2606_07156_amd as amp
    from amp_data.synth import WORKLOADS, draw_k, make_queries

    dev = torch.device("cuda:0")
    w = WORKLOADS["serving"]
    if args.serve_n:
        w = w.scaled(n=args.serve_n)
    t = time.perf_counter()
    b16 = serving_base_on_device(w, dev)
    torch.cuda.synchronize()
    log(f"[c5] generated {b16.shape} bf16 corpus in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    h = amp.amp_index_build(b16, w.nlist, w.M, iters=20, seed=w.seed, metric="ip", grid_kind=w.grid_kind)
    arr = amp.amp_index_get_arrays(h)
    sizes = np.diff(arr["list_offsets"]).astype(np.int64)
    args.idx_sizes = sizes
    log(f"[c5] built IVF{w.nlist}/PQ{w.M} on the device in {time.perf_counter() - t:.1f}s; list sizes "
        f"min/mean/max {sizes.min()}/{sizes.mean():.0f}/{sizes.max()}, grid_e {arr['grid_e']}")
    t = time.perf_counter()
    TQ = make_queries(w, args.train_queries, train=True)
    allowed = tuple(int(b) for b in args.allowed.split(","))
    rep = amp.amp_index_train_predictor(h, TQ, 10, 64, gamma=args.gamma, epsilon=args.epsilon, C_=args.svr_c,
                                        n_samples=1280, allowed=allowed)
    model = amp.amp_index_get_predictor(h)
    log(f"[c5] trained predictor in {time.perf_counter() - t:.1f}s: {rep}")
    nq = args.nq or 4096
    Q = make_queries(w, nq)  # bf16-representable rows
    Qb = np.ascontiguousarray((Q.view(np.uint32) >> 16).astype(np.uint16))
    r = np.random.Generator(np.random.PCG64([w.seed, 9002]))
    kq = np.array([10, 50, 100], np.int32)[r.integers(0, 3, nq)]
    npq = np.array([16, 64, 256], np.int32)[r.integers(0, 3, nq)]
    t = time.perf_counter()
    truth = exact_ip_bf16(b16, Q, 10, dev) if args.recall else None
    log(f"[c5] exact inner-product top-10 of {nq} queries in {time.perf_counter() - t:.1f}s")
    qdev = torch.from_numpy(Qb.view(np.int16)).to(dev)
    pols = policy_list(args.policies, allowed)
    apply_schedule(amp, h, args, allowed, nq)
    res = measure(h, w, Qb, kq, npq, pols, args, truth, "c5", qdev=qdev, q_dtype="bf16")
    head = "adaptive" if "adaptive" in res else next(iter(res))
    rh = res[head]
    fp = res.get("fp32")
    # serving: one Poisson arrival rate through the serving loop
    srv = serve_once(h, Qb, kq, npq, args.serve_rate, args.serve_seconds, head, args.serve_batch) \
        if args.serve_rate > 0 else None
    if srv:
        log(f"[c5] serving {srv}")
    gran = measure_granularity(h, w, Qb, kq, npq, truth, args, TQ, 10, 64, allowed, "c5", qdev=qdev,
                               q_dtype="bf16") if args.granularity else None
    del b16
    line = {
        "metric": "QPS at recall@10 (adaptive vs full-precision, same GPU); p99 latency",
        "value": round(rh["qps"], 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(rh["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32" if head != "fp32" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n}x{w.d} bf16 unit-normalised mixture ({w.n_comp} components), "
                               f"inner product, IVF{w.nlist}/PQ{w.M}x256 built on the device, {nq} BF16 queries "
                               "per step, per-query k in {10,50,100} and nprobe in {16,64,256}",
                   "policy": head, "launch": "HIP graph replay, per-query sizes on the device",
                   "recall_at_10": round(rh["recall10"], 4) if rh["recall10"] is not None else None,
                   "recall_definition": f"10-recall@10 over all {nq} queries against exact FP64 inner-product "
                                        "search of the BF16 corpus; 1-recall@10 in policies",
                   "speedup_vs_fp32": round(rh["qps"] / fp["qps"], 3) if fp else None,
                   "recall_ratio_vs_fp32": round(rh["recall10"] / max(fp["recall10"], 1e-9), 4)
                   if fp and rh["recall10"] is not None else None,
                   "bits_share": rh["bits"],
                   "predictor": {kk: rep[kk] for kk in ("n_sv", "label_hist", "n_pairs")},
                   "policies": summary(res),
                   "granularity_subspace": gran,
                   "serving": srv},
        "mfma": mfma_of(rh, w, nq),
        "roofline": roofline_of(rh, w, nq, TRAFFIC_FILE_C5),
    }
    if not args.no_cpu:
        kw = dict(dict(pols)[head])
        if head == "adaptive":
            kw["model"] = model
        arr.pop("list_sizes", None)
        arr["list_sizes"] = sizes.astype(np.int32)
        line["cpu_baseline"] = cpu_baseline(arr, Q, kq, npq, kw, budget_s=args.cpu_budget)
        log(f"[c5] cpu baseline {line['cpu_baseline']}")
    del arr
    h.free()
    if args.secondary:
        line["config"]["secondary"] = secondary_mid(args)
    print(json.dumps(line), flush=True)


def secondary_mid(args):
    """The mid-size workload (1M x 128 integer data, IVF1024 / PQ16, 10 000
    queries, nprobe 32, k 10) measured the same way: adaptive, FP32 and
    fixed 16-bit QPS with recall over all queries."""
    import paper_2606_07156_amd as amp
    from amp_data.synth import make_queries
    from amp_data.workloads import load_or_build

    w, base, idx = load_or_build("mid", args.cache_dir, log=lambda m: log("[c2] " + m))
    Q = make_queries(w)
    h = amp.amp_index_from_arrays(idx)
    amp.amp_index_to_device(h, 0)
    t = time.perf_counter()
    truth = exact_knn_device(base, Q, w.k, w.metric)
    log(f"[c2] exact kNN of {len(Q)} queries in {time.perf_counter() - t:.1f}s")
    TQ = make_queries(w, args.train_queries, train=True)
    rep = amp.amp_index_train_predictor(h, TQ, w.k, w.nprobe, gamma=args.gamma, epsilon=args.epsilon,
                                        C_=args.svr_c, n_samples=1280)
    args.idx_sizes = idx["list_sizes"].astype(np.int64)
    res = measure(h, w, Q, w.k, w.nprobe, policy_list("adaptive,fp32,fixed16", (4, 8, 12, 16)), args, truth, "c2")
    ra, rf = res["adaptive"], res["fp32"]
    out = {"workload": f"{w.name}: {w.n}x{w.d} integer-valued Gaussian mixture ({w.n_comp} components), l2, "
                       f"IVF{w.nlist}/PQ{w.M}x256, {len(Q)} queries per step, nprobe {w.nprobe}, k {w.k}",
           "qps": round(ra["qps"], 1), "speedup_vs_fp32": round(ra["qps"] / rf["qps"], 3),
           "recall_definition": f"1- and 10-recall@10 over all {len(Q)} queries against exact FP64 kNN",
           "policies": summary(res), "roofline": roofline_of(ra, w, len(Q), TRAFFIC_FILE),
           "mfma": mfma_of(ra, w, len(Q)), "predictor": {kk: rep[kk] for kk in ("n_sv", "label_hist")}}
    if args.granularity:
        out["granularity_subspace"] = measure_granularity(h, w, Q, w.k, w.nprobe, truth, args, TQ, w.k, w.nprobe,
                                                          (4, 8, 12, 16), "c2")
    if args.cl_slices > 0:
        out["cl"] = measure_cl(h, w, Q, truth, args, ra)
    return out


def measure_granularity(h, w, Q, kq, npq, truth, args, TQ, k_train, np_train, allowed, tag, qdev=None,
                        q_dtype=None):
    """The adaptive policy with a width per (pair, subspace) in the quantiser
    (the pair's lane budget shared by its subspaces), its predictor retrained
    for that quantiser; the per-pair predictor is restored afterwards."""
    import paper_2606_07156_amd as amp
    saved = amp.amp_index_get_predictor(h)
    rep = amp.amp_index_train_predictor(h, TQ, k_train, np_train, gamma=args.gamma, epsilon=args.epsilon,
                                        C_=args.svr_c, n_samples=1280, allowed=allowed, granularity="subspace")
    log(f"[{tag}] predictor for per-subspace widths: {rep}")
    res = measure(h, w, Q, kq, npq, [("adaptive_sub", dict(policy="adaptive", allowed=allowed,
                                                           granularity="subspace"))],
                  args, truth, tag, qdev=qdev, q_dtype=q_dtype)
    amp.amp_index_set_predictor(h, saved)
    return {"predictor": {kk: rep[kk] for kk in ("n_sv", "label_hist")}, "policies": summary(res)}


def measure_cl(h, w, Q, truth, args, r_fp32cl):
    """Cluster locating on 8-bit codes: the sub-space map (S slices, P
    sub-spaces per slice) and the CL predictor (gamma 0.1, C 10) on training
    queries, then the adaptive LUT policy with integer CL at 8 bits and with
    adaptive CL widths (low width 4): CL stage time (codes, predictor,
    distances), share of partial distances at the low width, recall."""
    import paper_2606_07156_amd as amp
    from amp_data.synth import make_queries
    t = time.perf_counter()
    amp.amp_index_build_cl_map(h, args.cl_slices, args.cl_subspaces, iters=20, seed=w.seed)
    t_map = time.perf_counter() - t
    TQ = make_queries(w, args.train_queries, train=True)
    t = time.perf_counter()
    rep = amp.amp_index_train_cl_predictor(h, TQ, w.nprobe, low=4, n_samples=1280, gamma=0.1, C_=10.0,
                                           epsilon=args.cl_epsilon)
    log(f"[cl] map S={args.cl_slices} P={args.cl_subspaces} in {t_map:.1f}s; CL predictor in "
        f"{time.perf_counter() - t:.1f}s: {rep}")
    allowed = (4, 8, 12, 16)
    pols = [("adaptive_cl8", dict(policy="adaptive", allowed=allowed, cl_policy="fixed", cl_bits=8)),
            ("adaptive_clA", dict(policy="adaptive", allowed=allowed, cl_policy="adaptive", cl_bits=4))]
    a = argparse.Namespace(**vars(args))
    a.autotune = 0
    res = measure(h, w, Q, w.k, w.nprobe, pols, a, truth, "cl")
    return {"slices": args.cl_slices, "subspaces_per_slice": args.cl_subspaces,
            "predictor": {kk: rep[kk] for kk in ("n_sv", "label_hist", "n_pairs")},
            "fp32_cl_ms": round(r_fp32cl["stages"]["cl"], 4),
            "policies": summary(res)}


def single(args):
    """One named workload with constant k and nprobe (profiling runs: the mid
    workload, the streaming regime with --replicate, the high-dimensional
    workload with --gpu-build)."""
    import torch

    import paper_2606_07156_amd as amp
    from amp_data.synth import make_queries
    from amp_data.workloads import load_or_build

    if args.gpu_build:
        from amp_data.synth import WORKLOADS, make_base
        w = WORKLOADS[args.workload]
        t = time.perf_counter()
        base = make_base(w)
        log(f"[bench] generated base {base.shape} in {time.perf_counter() - t:.1f}s")
        t = time.perf_counter()
        hb = amp.amp_index_build(base, w.nlist, w.M, iters=20, seed=w.seed, integer_data=w.integer_data,
                                 grid_kind=w.grid_kind, metric=w.metric)
        idx = amp.amp_index_get_arrays(hb)
        del hb
        log(f"[bench] built IVF{w.nlist}/PQ{w.M} on the device in {time.perf_counter() - t:.1f}s")
    else:
        w, base, idx = load_or_build(args.workload, args.cache_dir, log=lambda m: log("[bench] " + m))
    if args.nq:
        w = w.scaled(nq=args.nq)
    streaming = args.replicate > 1
    if streaming:
        from amp_data.workloads import replicate
        import dataclasses
        idx = replicate(idx, args.replicate)
        w = dataclasses.replace(w, n=w.n * args.replicate)
        log(f"[bench] replicated every list {args.replicate}x: {len(idx['ids'])} vectors, "
            f"{idx['codes'].nbytes / 1e6:.0f} MB of codes")
    Q = make_queries(w)
    h = amp.amp_index_from_arrays(idx)
    amp.amp_index_to_device(h, 0)
    if streaming:
        truth = np.zeros((len(Q), w.k), np.int64)  # duplicates tie: recall is not meaningful here
    elif not args.recall:
        truth = None
    else:
        t = time.perf_counter()
        truth = exact_knn_device(base, Q, w.k, w.metric)
        log(f"[bench] exact kNN of {len(Q)} queries in {time.perf_counter() - t:.1f}s")
    allowed = tuple(int(b) for b in args.allowed.split(","))
    TQ = make_queries(w, args.train_queries, train=True)
    rep = amp.amp_index_train_predictor(h, TQ, w.k, w.nprobe, gamma=args.gamma, epsilon=args.epsilon,
                                        allowed=allowed, C_=args.svr_c, n_samples=1280)
    model = amp.amp_index_get_predictor(h)
    log(f"[bench] trained predictor: {rep}")
    apply_schedule(amp, h, args, allowed, len(Q))
    args.idx_sizes = idx["list_sizes"].astype(np.int64)
    pols = policy_list(args.policies, allowed)
    res = measure(h, w, Q, w.k, w.nprobe, pols, args, truth, "bench")
    head = "adaptive" if "adaptive" in res else next(iter(res))
    rh = res[head]
    fp = res.get("fp32")
    line = {
        "metric": "QPS at recall@10 (adaptive vs full-precision, same GPU); p99 latency",
        "value": round(rh["qps"], 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(rh["ms"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32" if head != "fp32" else "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n}x{w.d} {KIND_TEXT.get(w.kind, w.kind)} ({w.n_comp} components), "
                               f"{w.metric}, IVF{w.nlist}/PQ{w.M}x256, {len(Q)} queries per step, nprobe "
                               f"{w.nprobe}, k {w.k}" + (", index built on the device" if args.gpu_build else "")
                               + (f"; every list replicated {args.replicate}x (streaming regime)"
                                  if streaming else ""),
                   "policy": head, "recall_at_10": round(rh["recall10"], 4) if rh["recall10"] is not None else None,
                   "speedup_vs_fp32": round(rh["qps"] / fp["qps"], 3) if fp else None,
                   "policies": summary(res)},
        "mfma": mfma_of(rh, w, len(Q)),
        "roofline": roofline_of(rh, w, len(Q), STREAM_TRAFFIC_FILE if streaming else TRAFFIC_FILE),
    }
    if not args.no_cpu and not streaming:
        kw = dict(dict(pols)[head])
        if head == "adaptive":
            kw["model"] = model
        line["cpu_baseline"] = cpu_baseline(idx, Q, w.k, w.nprobe, kw, budget_s=args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
