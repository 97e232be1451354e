"""Throughput benchmark of the adaptive-precision IVF-PQ search on one MI355X.

A step is one search of the whole query batch of the mid-size workload
(1M x 128 integer-valued vectors from a 1024-component Gaussian mixture,
IVF1024 / PQ16x256, 10 000 queries, nprobe 32, k 10): coarse distances,
probe selection, precision prediction, work queue, LUT build + quantisation
+ scan, top-k merge.  Queries and the index are resident in HBM before the
timed region.  Prints one JSON line (see the fields below); a per-policy
table goes to stderr.
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
STREAM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_scan_stream_traffic.json")


def _kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "amp_internal.h"):
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
    idx, Q, k, nprobe, kw = args
    t = time.perf_counter()
    oracle.search(idx, Q, k, nprobe, **kw)
    return time.perf_counter() - t


def cpu_baseline(idx, Q, k, nprobe, kw, budget_s=20.0):
    """Time the oracle on a bounded sample of the same queries, one worker
    process per host core."""
    cores = os.cpu_count() or 1
    cores = min(cores, 16)
    t0 = time.perf_counter()
    _cpu_worker((idx, Q[:2], k, nprobe, kw))
    per_q = max((time.perf_counter() - t0) / 2, 1e-4)
    n = int(min(len(Q), max(cores, budget_s * cores / per_q)))
    n = max(cores, (n // cores) * cores)
    chunks = [(idx, Q[i::cores][: n // cores], k, nprobe, kw) for i in range(cores)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_cpu_worker, chunks)
    wall = time.perf_counter() - t0
    return dict(value=n / wall, unit="queries/s", cores=cores, kind="oracle",
                sample=f"first {n} of {len(Q)} queries (interleaved over {cores} processes), "
                       f"{wall:.1f} s wall")


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
    dev = torch.device("cuda:0")
    qd = torch.from_numpy(Q).to(dev)
    stream = torch.cuda.Stream()
    rows = []
    for B in [int(b) for b in args.batches.split(",")]:
        for pol in ("adaptive", "fp32"):
            kw = dict(policy=pol)
            e = amp.amp_index_autotune(h, Q[:B], 10, NP[:B], repeats=3, **kw)
            out = dict(ids=torch.empty((B, 10), dtype=torch.int64, device=dev),
                       dist=torch.empty((B, 10), dtype=torch.float32, device=dev))
            reps = max(3, min(200, int(2000 / max(B, 1)) + 3))
            for i in range(2):
                amp.amp_search(h, qd[:B], 10, NP[:B], out=out, stream=stream, **kw)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for i in range(reps):
                amp.amp_search(h, qd[:B], 10, NP[:B], out=out, stream=stream, **kw)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            rows.append(dict(batch=B, policy=pol, ms=round(ms, 4), qps=round(B / ms * 1e3, 1),
                             schedule={kk: e[kk] for kk in ("chunk", "chunk1", "narrow", "lut_dtype", "queue")},
                             tuned_ms=round(e["ms"], 4), automatic_ms=round(e["ms_default"], 4)))
            log(f"[sweep] B={B:5d} {pol:8s} {ms:8.3f} ms/batch {B / ms * 1e3:11.0f} QPS  schedule "
                f"{rows[-1]['schedule']} (tuned {e['ms']:.3f} ms vs automatic {e['ms_default']:.3f} ms)")
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
    ap.add_argument("--workload", default="mid")
    ap.add_argument("--nq", type=int, default=0)
    ap.add_argument("--policies", default="adaptive,fp32,fixed16,fixed8,fixed4")
    ap.add_argument("--train-queries", type=int, default=256)
    ap.add_argument("--gamma", type=float, default=10.0)
    ap.add_argument("--epsilon", type=float, default=0.1)
    ap.add_argument("--svr-c", type=float, default=1.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--recall-queries", type=int, default=200,
                    help="queries checked against exact kNN (0: skip; profiling runs)")
    ap.add_argument("--cache-dir", default="/tmp/amp_bench_cache")
    ap.add_argument("--replicate", type=int, default=0,
                    help="R > 1: every list R times larger (working set beyond the last-level cache; "
                         "use with a small --nq for the streaming regime)")
    ap.add_argument("--graph", type=int, default=1,
                    help="1: timed searches replay a captured HIP graph (0: plain launches)")
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
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="arrival window per rate")
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
              "note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2606_07156_amd as amp
    from amp_data.synth import make_queries
    from amp_data.workloads import load_or_build

    if args.gpu_build:
        # large workloads: index built on the device by the library's builder
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
    if args.replicate > 1:
        # streaming regime: every list `replicate` times larger, no recall
        from amp_data.workloads import replicate
        import dataclasses
        idx = replicate(idx, args.replicate)
        w = dataclasses.replace(w, n=w.n * args.replicate)
        args.recall_queries = 0
        args.no_cpu = True
        log(f"[bench] replicated every list {args.replicate}x: {len(idx['ids'])} vectors, "
            f"{idx['codes'].nbytes / 1e6:.0f} MB of codes")
    log(f"[bench] list sizes min/mean/max {idx['list_sizes'].min()}/{idx['list_sizes'].mean():.0f}/"
        f"{idx['list_sizes'].max()}")
    Q = make_queries(w)
    h = amp.amp_index_from_arrays(idx)
    amp.amp_index_to_device(h, 0)
    dev = torch.device("cuda:0")
    qd = torch.from_numpy(Q).to(dev)
    nq, k, nprobe = len(Q), w.k, w.nprobe
    # streaming regime: every search takes a fresh batch from a pool (no code
    # reuse between consecutive searches); plain launches (the query pointer
    # changes)
    n_batches = args.steps + args.warmup if args.replicate > 1 else 1
    if n_batches > 1:
        args.graph = 0
        QP = make_queries(w.scaled(nq=nq * n_batches), nq * n_batches)
        qpool = torch.from_numpy(QP).to(dev)
        batch = lambda i: qpool[(i % n_batches) * nq:(i % n_batches + 1) * nq]
    else:
        batch = lambda i: qd
    out = dict(ids=torch.empty((nq, k), dtype=torch.int64, device=dev),
               dist=torch.empty((nq, k), dtype=torch.float32, device=dev),
               qdist=torch.empty((nq, k), dtype=torch.int64, device=dev))
    out_probes = torch.empty((nq, nprobe), dtype=torch.int32, device=dev)
    out_bits = torch.empty((nq, nprobe), dtype=torch.uint8, device=dev)
    # a created stream (default priority): graph capture needs one
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()

    # exact ground truth for recall@10 on a sample of queries (FP64 brute force)
    import oracle
    nr = min(args.recall_queries, nq)
    t = time.perf_counter()
    if nr and base.shape[0] * base.shape[1] > 2e8:
        truth = exact_knn_device(base, Q[:nr], k, w.metric)  # FP64 on the device
    else:
        truth = oracle.exact_knn(base, Q[:nr], k, w.metric) if nr else None
    log(f"[bench] exact kNN of {nr} queries in {time.perf_counter() - t:.1f}s")

    allowed = tuple(int(b) for b in args.allowed.split(","))
    # precision predictor fitted on a disjoint training query stream
    t = time.perf_counter()
    TQ = make_queries(w, args.train_queries, train=True)
    rep = amp.amp_index_train_predictor(h, TQ, k, nprobe, gamma=args.gamma, epsilon=args.epsilon, allowed=allowed,
                                        C_=args.svr_c, n_samples=1280)
    model = amp.amp_index_get_predictor(h)
    log(f"[bench] trained predictor in {time.perf_counter() - t:.1f}s: {rep}")

    pols = []
    for p in args.policies.split(","):
        if p == "fp32":
            pols.append(("fp32", dict(policy="fp32")))
        elif p == "adaptive":
            pols.append(("adaptive", dict(policy="adaptive", allowed=allowed)))
        elif p.startswith("fixed"):
            pols.append((p, dict(policy="fixed", bits=int(p[5:]))))
    results = {}
    # algorithmic bytes of the scan: one read of each probed list's codes per pair
    sizes = idx["list_sizes"].astype(np.int64)
    tuned = {}
    for name, kw in pols:
        if args.schedule:
            # a fixed schedule for every policy (profiling runs: no tuning trials in the trace)
            f = [int(x) for x in args.schedule.split(",")]
            c, c1, nw, lt = f[:4]
            ent = dict(policy_kind=amp.POLICIES[kw["policy"]], chunk=c, chunk1=c1, narrow=nw, lut_dtype=lt,
                       queue=f[4] if len(f) > 4 else 0)
            lg = int(np.ceil(np.log2(nq)))
            amp.amp_index_set_tuning(h, [dict(ent, nq_log2=lg)])
            tuned[name] = dict(ent, ms=0.0, ms_default=0.0)
        elif args.autotune:
            # schedule (unit chunking, LUT row width, LC dtype) timed for this
            # batch shape; results do not depend on it
            tuned[name] = amp.amp_index_autotune(h, QP[:nq] if n_batches > 1 else Q, k, nprobe, repeats=3, **kw)
            log(f"[bench] {name}: autotuned schedule {tuned[name]}")
        out["probes"], out["bits"] = (None, None) if nr else (out_probes, out_bits)
        for i in range(args.warmup):
            amp.amp_search(h, batch(args.steps + i), k, nprobe, out=out, stream=stream, graph=args.graph, **kw)
        torch.cuda.synchronize()
        # timed region: K searches enqueued back to back on one stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(args.steps):
            amp.amp_search(h, batch(i), k, nprobe, out=out, stream=stream, graph=args.graph, **kw)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        # stage breakdown and per-batch latency: separate, synchronised searches
        stages, lat, works = [], [], []
        for i in range(args.steps):
            o = amp.amp_search(h, batch(i), k, nprobe, out=out, stream=stream, stage_ms=True, work=True, **kw)
            stages.append(o["stage_ms"])
            lat.append(o["stage_ms"]["total"])
            works.append(o["work"])
        if nr:
            g = amp.amp_search(h, Q[:nr], k, nprobe, want_probes=True, want_bits=True, **kw)
            rec1 = oracle.recall_1_at(g["ids"], truth)
            rec10 = oracle.recall_at(g["ids"], truth)
        else:
            # outputs of the last timed search (device), no recall
            g = dict(probes=out_probes.cpu().numpy(), bits=out_bits.cpu().numpy())
            rec1 = rec10 = float("nan")
        pr = g["probes"]
        bits = g["bits"][pr >= 0]
        hist = {int(b): round(float((bits == b).mean()), 4) for b in np.unique(bits)}
        scale = nq / len(pr)
        code_bytes = float(sizes[pr[pr >= 0]].sum()) * w.M * scale
        # the phase-2 scan's own counters: code bytes of the (query, list)
        # pairs it scanned, live and skipped pairs (a pair whose LUT base
        # exceeds its query's bound is skipped whole after LUT pass 1)
        wk = {kk: float(np.mean([x[kk] for x in works])) for kk in works[0]}
        n_pairs_all = wk["live_pairs"] + wk["dead_pairs"]
        # algorithmic work per launch = per-pair figure x pairs processed:
        # every probed pair's LUT (256 M entries) and its list's lookup-adds
        # (n M), whether the bound test let it skip the scan or not
        scan_ops = (float(sizes[pr[pr >= 0]].sum()) + 256.0 * (pr >= 0).sum()) * w.M * scale
        exec_ops = wk["scan_bytes"] + 256.0 * w.M * n_pairs_all
        st = {s: float(np.mean([x[s] for x in stages])) for s in stages[0]}
        results[name] = dict(qps=nq / (ms / 1e3), ms=ms, recall1=rec1, recall10=rec10, stages=st,
                             code_bytes=code_bytes, scan_ops=scan_ops, exec_ops=exec_ops, scan_bytes=wk["scan_bytes"],
                             live_pairs=wk["live_pairs"], dead_pairs=wk["dead_pairs"], bits=hist,
                             p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)))
        log(f"[bench] {name:8s} {ms:8.3f} ms/step  {nq / ms * 1e3:12.0f} QPS  1-recall@10 {rec1:.4f}  "
            f"10-recall@10 {rec10:.4f}  bits {hist}  " + " ".join(f"{s}={v:.3f}" for s, v in st.items()))

    head = "adaptive" if "adaptive" in results else next(iter(results))
    r = results[head]
    scan_ms = r["stages"]["scan2"]
    # algorithmic work of the phase-2 scan: per (query, probed list) pair one
    # LUT entry per (subspace, codeword) and one lookup-add per (vector,
    # subspace); "executed" counts only what ran (pairs skipped whole after
    # the LUT's first pass scan nothing)
    achieved = r["scan_ops"] / (scan_ms / 1e3) / 1e12
    executed = r["exec_ops"] / (scan_ms / 1e3) / 1e12
    streaming = args.replicate > 1
    mix = head in ("adaptive",)
    kname = ("k_scan_mix<M,2,1,NR>: phase-2 scan, every lane class in one launch" if mix else
             "k_scan<LW,M,2,1,NR>: phase-2 scan of the policy's lane class")
    traffic = measured_traffic(STREAM_TRAFFIC_FILE if streaming else TRAFFIC_FILE)
    work = {"live_pairs": round(r["live_pairs"]), "skipped_pairs": round(r["dead_pairs"]),
            "scanned_code_bytes": round(r["scan_bytes"]), "probed_code_bytes": round(r["code_bytes"])}
    if streaming:
        # no cross-query reuse of codes: a scan of every probed pair's codes
        # would be bounded by HBM bandwidth; algorithmic bytes = each probed
        # list's codes once per pair; "executed" = the bytes of the pairs the
        # scan read (the rest were skipped by the bound test)
        gbs = r["code_bytes"] / (scan_ms / 1e3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                    "kernel_ms": round(scan_ms, 4), "algorithmic_bytes_per_launch": round(r["code_bytes"]),
                    "executed": {"bytes_per_launch": round(r["scan_bytes"]),
                                 "GB/s": round(r["scan_bytes"] / (scan_ms / 1e3) / 1e9, 1)},
                    "work": work}
    else:
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                    "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": traffic, "kernel": kname,
                    "kernel_ms": round(scan_ms, 4), "algorithmic_ops_per_launch": round(r["scan_ops"]),
                    "executed": {"ops_per_launch": round(r["exec_ops"]), "TOP/s": round(executed, 3),
                                 "frac": round(executed / ALU_PEAK_TOPS, 4)},
                    "work": work}
    fp = results.get("fp32")
    # the two dense contractions on MFMA: CL (FP32 MFMA) and the LUT build
    # (BF16 MFMA, fused into the scan kernels: rate over the scan stages, a
    # lower bound on its own utilisation)
    st_h = r["stages"]
    n_pairs = float(nq) * nprobe
    cl_flops = 2.0 * nq * w.nlist * w.d
    lc_flops = n_pairs * 2.0 * 256 * w.d
    cl_tf = cl_flops / (st_h["cl"] / 1e3) / 1e12
    lc_tf = lc_flops / ((st_h["scan1"] + st_h["scan2"]) / 1e3) / 1e12
    mfma_use = {"cl": {"flop_per_search": cl_flops, "tflops": round(cl_tf, 2), "peak": FP32_MFMA_TFLOPS,
                       "frac": round(cl_tf / FP32_MFMA_TFLOPS, 4)},
                "lc": {"flop_per_search": lc_flops, "tflops_over_scan": round(lc_tf, 2), "peak": BF16_MFMA_TFLOPS,
                       "frac": round(lc_tf / BF16_MFMA_TFLOPS, 4)}}
    # end-to-end QPS against reading every probed list's codes once per query
    # from HBM (no reuse) at peak bandwidth
    bytes_per_q = r["code_bytes"] / nq
    hbm_q = HBM_PEAK_GBS * 1e9 / bytes_per_q
    hbm_bound = {"code_bytes_per_query": round(bytes_per_q), "qps_at_hbm_peak": round(hbm_q),
                 "frac": round(r["qps"] / hbm_q, 4)}
    line = {
        "metric": "QPS at recall@10 (adaptive vs full-precision, same GPU); p99 latency",
        "value": round(r["qps"], 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32" if head != "fp32" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n}x{w.d} {KIND_TEXT.get(w.kind, w.kind)} ({w.n_comp} components), "
                               f"{w.metric}, IVF{w.nlist}/PQ{w.M}x256, {nq} queries per step, nprobe {nprobe}, k {k}"
                               + (", index built on the device" if args.gpu_build else "")
                               + (f"; every list replicated {args.replicate}x (streaming regime)"
                                  if args.replicate > 1 else ""),
                   "policy": head,
                   "launch": "HIP graph replay" if args.graph else "kernel launches",
                   "schedule": ({kk: tuned[head][kk] for kk in ("chunk", "chunk1", "narrow", "lut_dtype", "queue", "ms",
                                                                "ms_default")} if head in tuned else "automatic"),
                   "recall_at_10": round(r["recall1"], 4),
                   "recall_definition": "1-recall@10 (exact nearest neighbour within the 10 returned); "
                                        f"10-recall@10 {r['recall10']:.4f}; {nr} queries vs FP64 brute force",
                   "speedup_vs_fp32": round(r["qps"] / fp["qps"], 3) if fp else None,
                   "recall_vs_fp32": round(r["recall1"] - fp["recall1"], 4) if fp else None,
                   "bits_share": r["bits"],
                   "batch_latency_ms_p50_p99": [round(r["p50"], 4), round(r["p99"], 4)],
                   "predictor": {kk: rep[kk] for kk in ("n_sv", "label_hist", "n_pairs")},
                   "policies": {n: {"qps": round(x["qps"], 1), "recall_at_10": round(x["recall1"], 4),
                                    "10_recall_at_10": round(x["recall10"], 4), "ms": round(x["ms"], 4),
                                    "scan_ms": round(x["stages"]["scan2"], 4)}
                                for n, x in results.items()}},
        "mfma": mfma_use,
        "hbm_bound": hbm_bound,
        "roofline": roofline,
    }
    if not args.no_cpu:
        kw = dict(pols)[head]
        if head == "adaptive":
            kw = dict(kw, model=model)
        line["cpu_baseline"] = cpu_baseline(idx, Q, k, nprobe, kw)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
