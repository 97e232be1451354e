"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  Integer policies: ids, integer distances and float
distances bit-exact (given the probe set, whose differences must be certified
FP32 near-ties).  FP32 policy and coarse distances: within the FP32 bounds
stated in tests/_parity.py (at most 1e-3 relative)."""
import os

import numpy as np
import pytest

import oracle
import paper_2606_07156_amd as amp
from amp_data import build_index, lossless_index, random_model
from amp_data.synth import WORKLOADS, make_base, make_queries
from _parity import certify_probes, check_coarse, compare_fp32, compare_integer

pytestmark = pytest.mark.gpu


def _ctx(idx, Q, base=None):
    h = amp.amp_index_from_arrays(idx)
    amp.amp_index_to_device(h, 0)
    return dict(idx=idx, Q=Q, base=base, h=h)


@pytest.fixture(scope="module")
def tiny():
    w = WORKLOADS["tiny"]
    base = make_base(w)
    idx = build_index(base, w.nlist, w.M, iters=10, seed=w.seed)
    return _ctx(idx, make_queries(w, 100), base)


@pytest.fixture(scope="module")
def midint():
    # the mid-size workload's shape (d=128, M=16, integer data) at a size the
    # oracle finishes in seconds
    w = WORKLOADS["mid"].scaled(n=60_000, nq=48, nlist=128)
    base = make_base(w)
    idx = build_index(base, w.nlist, w.M, iters=8, seed=w.seed, integer_data=True)
    return _ctx(idx, make_queries(w, 48), base)


def _gpu(ctx, k, nprobe, **pol):
    return amp.amp_search(ctx["h"], ctx["Q"], k, nprobe, want_probes=True, want_bits=True,
                          want_coarse=True, **pol)


def _oracle(ctx, k, nprobe, g, **pol):
    return oracle.search(ctx["idx"], ctx["Q"], k, nprobe, probes=g["probes"], **pol)


def test_coarse_distances_and_probe_sets(tiny):
    g = _gpu(tiny, 10, 8)
    check_coarse(g["coarse"], tiny["idx"], tiny["Q"])
    ties = certify_probes(g["probes"], tiny["idx"], tiny["Q"], 8)
    assert ties <= 2


@pytest.mark.parametrize("bits", [4, 8, 12, 16])
def test_fixed_width_is_bit_exact(tiny, bits):
    g = _gpu(tiny, 10, 8, policy="fixed", bits=bits)
    certify_probes(g["probes"], tiny["idx"], tiny["Q"], 8)
    ref = _oracle(tiny, 10, 8, g, policy="fixed", bits=bits)
    assert (g["bits"] == bits).all()
    compare_integer(g, ref)


def test_fp32_policy_within_fp32_bound(tiny):
    g = _gpu(tiny, 10, 8, policy="fp32")
    ref = _oracle(tiny, 10, 8, g, policy="fp32")
    assert (g["qdist"] == -1).all()
    swaps = compare_fp32(g, ref, tiny["idx"], tiny["Q"])
    assert swaps <= 3


def test_explicit_widths_are_bit_exact(tiny):
    r = np.random.default_rng(3)
    xb = r.choice(np.array([4, 8, 12, 16], np.uint8), size=(len(tiny["Q"]), 8))
    g = _gpu(tiny, 10, 8, policy="explicit", explicit_bits=xb)
    assert np.array_equal(g["bits"], xb)
    ref = _oracle(tiny, 10, 8, g, policy="explicit", explicit_bits=xb)
    compare_integer(g, ref)


@pytest.mark.parametrize("policy", ["explicit", "fixed"])
def test_stealing_unit_queue_is_bit_exact(tiny, policy):
    # the scan kernels' work-stealing queue (one range of units per XCD)
    # forced through the tuning table: same results as the oracle
    r = np.random.default_rng(5)
    nq = len(tiny["Q"])
    xb = r.choice(np.array([4, 8, 12, 16], np.uint8), size=(nq, 8)) if policy == "explicit" else None
    kw = dict(policy="explicit", explicit_bits=xb) if xb is not None else dict(policy="fixed", bits=8)
    amp.amp_index_set_tuning(tiny["h"], [dict(policy_kind=amp.POLICIES[policy], nq_log2=int(np.ceil(np.log2(nq))),
                                              chunk=256, chunk1=256, narrow=-1, lut_dtype=0, queue=1)])
    try:
        g = _gpu(tiny, 10, 8, **kw)
    finally:
        amp.amp_index_set_tuning(tiny["h"], [])
    ref = _oracle(tiny, 10, 8, g, **kw)
    compare_integer(g, ref)


def _dq2(idx, q, P):
    """d' of the probed lists of one query as the oracle forms it (squared
    grid residual; inner product: squared grid difference of query and
    centroid)."""
    inv = 2.0 ** -idx["grid_e"]
    out = []
    if idx["metric"] == "ip":
        _, ci = oracle.index_grid(idx)
        qi = oracle.grid(np.asarray(q, np.float64) * inv, idx["grid_kind"])
        for p in P:
            r = qi - ci[p]
            out.append(int((r * r).sum()))
    else:
        for p in P:
            r = oracle.grid(oracle.residual_f32(q, idx["centroids"][p]).astype(np.float64) * inv,
                            idx["grid_kind"])
            out.append(int((r * r).sum()))
    return np.asarray(out, dtype=np.int64)


def _spread_model(ctx, nprobe, seed=0, n_sv=200):
    """A seeded random regressor whose feature map covers the index's feature
    ranges and whose thresholds split the scores of these queries into four
    width classes (scores from the oracle)."""
    idx, Q = ctx["idx"], ctx["Q"]
    probes = [oracle.select_probes(oracle.coarse_distances(q, idx["centroids"], idx["metric"]), nprobe)
              for q in Q[:16]]
    dq = np.concatenate([_dq2(idx, q, P) for q, P in zip(Q[:16], probes)])
    feats = [dq, idx["radq"], idx["radq"], idx["list_sizes"], idx["list_sizes"]]
    lo, mul = [], []
    for f in feats:
        L = oracle.mitchell_log2_q8(np.asarray(f, dtype=np.int64))
        a, b = int(L.min()), int(L.max())
        lo.append(a)
        mul.append(int(1023 * 65536 // max(1, b - a)))
    m = random_model(seed, n_sv, lo, mul, gamma=1.0)
    ys = []
    for q, P in zip(Q[:16], probes):
        _, y = oracle.predict_pair_bits(_dq2(idx, q, P), P, idx["radq"], idx["list_sizes"], m)
        ys.extend(int(v) for v in y)
    m["theta"] = np.quantile(np.asarray(ys, dtype=np.float64), [0.25, 0.5, 0.75]).astype(np.int64)
    return m


def test_adaptive_predictor_and_search_are_bit_exact(tiny):
    m = _spread_model(tiny, 8)
    amp.amp_index_set_predictor(tiny["h"], m)
    g = _gpu(tiny, 10, 8, policy="adaptive")
    ref = _oracle(tiny, 10, 8, g, policy="adaptive", model=m)
    assert np.array_equal(g["bits"], ref["bits"].astype(np.uint8))
    assert len(np.unique(g["bits"])) >= 3
    compare_integer(g, ref)
    # restricted width sets and a score margin
    g2 = _gpu(tiny, 10, 8, policy="adaptive", allowed=(4, 8, 16), margin_q40=int(m["theta"][1] - m["theta"][0]))
    ref2 = _oracle(tiny, 10, 8, g2, policy="adaptive", model=m, allowed=(4, 8, 16),
                   margin_q40=int(m["theta"][1] - m["theta"][0]))
    assert np.array_equal(g2["bits"], ref2["bits"].astype(np.uint8))
    assert not (g2["bits"] == 12).any()
    compare_integer(g2, ref2)


@pytest.mark.parametrize("policy,bits", [("fixed", 4), ("fixed", 8), ("fixed", 12), ("fixed", 16), ("fp32", 0)])
def test_integer_data_exact_end_to_end(midint, policy, bits):
    """Integer data: coarse distances are exact in FP32, so probe sets must be
    identical with no near-tie allowance."""
    g = _gpu(midint, 10, 16, policy=policy, bits=bits)
    for i, q in enumerate(midint["Q"]):
        D64 = oracle.coarse_distances(q, midint["idx"]["centroids"])
        assert np.array_equal(g["coarse"][i].astype(np.float64), D64)
        assert np.array_equal(g["probes"][i], oracle.select_probes(D64, 16))
    ref = oracle.search(midint["idx"], midint["Q"], 10, 16, policy=policy, bits=bits)
    if policy == "fp32":
        compare_fp32(g, ref, midint["idx"], midint["Q"])
    else:
        compare_integer(g, ref)


def test_lut_build_is_exact_at_the_grid_extremes():
    """Codewords and residuals at the +-255 ends of the 9-bit grid: the
    largest LUT entries (8 * 510^2) and |ri|^2 + off terms the MFMA path must
    still reproduce exactly."""
    r = np.random.default_rng(21)
    nlist, M, dsub = 4, 16, 8
    d = M * dsub
    C = np.zeros((nlist, d), np.float32)
    C[1:] = r.choice([-255.0, 255.0], size=(nlist - 1, d))
    CB = r.choice([-255.0, 255.0, 0.0, 254.0, -1.0], size=(M, 256, dsub)).astype(np.float32)
    CB[:, :8] = 255.0
    CB[:, 8:16] = -255.0
    n_per = 300
    codes = r.integers(0, 256, size=(nlist * n_per, M)).astype(np.uint8)
    idx = dict(d=d, M=M, dsub=dsub, nlist=nlist, ksub=256, metric="l2", grid_kind="u9", grid_e=0,
               centroids=C, codebook=CB, list_offsets=np.arange(0, nlist * n_per + 1, n_per),
               ids=np.arange(nlist * n_per, dtype=np.int64), codes=codes,
               list_sizes=np.full(nlist, n_per, np.int32), radq=np.full(nlist, 100, np.int32))
    Q = r.choice([-255.0, 255.0, 0.0], size=(12, d)).astype(np.float32)
    Q[:4] = 255.0
    Q[4:8] = -255.0
    ctx = _ctx(idx, Q)
    for bits in (16, 12, 4):
        g = _gpu(ctx, 20, 4, policy="fixed", bits=bits)
        ref = _oracle(ctx, 20, 4, g, policy="fixed", bits=bits)
        compare_integer(g, ref)


def test_edge_cases_padding_chunking_empty_lists_and_per_query_sizes(monkeypatch):
    idx, base = lossless_index(seed=9, nlist=10, M=8, dsub=4,
                               per_list=[0, 1, 257, 600, 3, 0, 1025, 64, 255, 9])
    r = np.random.default_rng(4)
    Q = r.integers(-40, 41, size=(37, 32)).astype(np.float32)
    ctx = _ctx(idx, Q, base)
    # k larger than every candidate set, nprobe = nlist, nq not a multiple of anything
    g = _gpu(ctx, 1024, 10, policy="fixed", bits=16)
    ref = _oracle(ctx, 1024, 10, g, policy="fixed", bits=16)
    compare_integer(g, ref)
    g = _gpu(ctx, 1024, 2, policy="fixed", bits=16)
    ref = _oracle(ctx, 1024, 2, g, policy="fixed", bits=16)
    compare_integer(g, ref)
    assert (g["ids"] == -1).any() and (g["qdist"][g["ids"] == -1] == np.iinfo(np.int64).max).all()
    # the lossless index at 16 bits with s = 0 reproduces exact kNN
    truth = oracle.exact_knn(base, Q, 10)
    g10 = _gpu(ctx, 10, 10, policy="fixed", bits=16)
    assert np.array_equal(g10["ids"], truth)
    # lists split into many work-unit chunks (ragged tails)
    monkeypatch.setenv("AMP_CHUNK", "100")
    for bits in (4, 16):
        g = _gpu(ctx, 7, 6, policy="fixed", bits=bits)
        compare_integer(g, _oracle(ctx, 7, 6, g, policy="fixed", bits=bits))
    gf = _gpu(ctx, 7, 6, policy="fp32")
    compare_fp32(gf, _oracle(ctx, 7, 6, gf, policy="fp32"), ctx["idx"], ctx["Q"])
    monkeypatch.delenv("AMP_CHUNK")
    # per-query k and nprobe
    kq = r.integers(1, 40, size=len(Q)).astype(np.int32)
    npq = r.integers(1, 11, size=len(Q)).astype(np.int32)
    g = _gpu(ctx, kq, npq, policy="fixed", bits=8)
    ref = _oracle(ctx, kq, npq, g, policy="fixed", bits=8)
    compare_integer(g, ref)
    # a single query
    g1 = amp.amp_search(ctx["h"], Q[:1], 5, 3)
    r1 = oracle.search(idx, Q[:1], 5, 3)
    compare_integer(g1, r1)


def test_results_do_not_depend_on_batch_composition(tiny):
    Q = tiny["Q"]
    full = amp.amp_search(tiny["h"], Q, 10, 8, policy="fixed", bits=4)
    for i in (0, 17, 99):
        one = amp.amp_search(tiny["h"], Q[i:i + 1], 10, 8, policy="fixed", bits=4)
        assert np.array_equal(one["ids"][0], full["ids"][i])
        assert np.array_equal(one["qdist"][0], full["qdist"][i])
    perm = np.random.default_rng(5).permutation(len(Q))
    shuf = amp.amp_search(tiny["h"], Q[perm], 10, 8, policy="fixed", bits=4)
    assert np.array_equal(shuf["ids"], full["ids"][perm])
    again = amp.amp_search(tiny["h"], Q, 10, 8, policy="fixed", bits=4)
    assert np.array_equal(again["ids"], full["ids"]) and np.array_equal(again["qdist"], full["qdist"])


def test_device_mode_matches_host_mode(tiny):
    torch = pytest.importorskip("torch")
    Q = tiny["Q"]
    host = amp.amp_search(tiny["h"], Q, 10, 8, policy="fixed", bits=8)
    qd = torch.from_numpy(Q).cuda()
    out = dict(ids=torch.empty((len(Q), 10), dtype=torch.int64, device="cuda"),
               dist=torch.empty((len(Q), 10), dtype=torch.float32, device="cuda"),
               qdist=torch.empty((len(Q), 10), dtype=torch.int64, device="cuda"))
    s = torch.cuda.current_stream()
    amp.amp_search(tiny["h"], qd, 10, 8, policy="fixed", bits=8, out=out, stream=s)
    torch.cuda.synchronize()
    assert np.array_equal(out["ids"].cpu().numpy(), host["ids"])
    assert np.array_equal(out["qdist"].cpu().numpy(), host["qdist"])


def _small(kind, metric="l2", grid_kind="u9", n=12_000, d=64, n_comp=48, nlist=32, M=16, seed=77, nq=40):
    from amp_data.synth import Workload
    w = Workload("t", n, d, n_comp, nq, nlist, M, 8, 10, kind, seed, metric=metric, grid_kind=grid_kind)
    base = make_base(w)
    idx = build_index(base, nlist, M, iters=8, seed=seed, grid_kind=grid_kind, metric=metric)
    return _ctx(idx, make_queries(w, nq), base)


@pytest.fixture(scope="module")
def ipctx():
    # unit-normalised clusters, inner product (the serving workload's metric)
    return _small("vmf", metric="ip", d=64, M=16)


@pytest.mark.parametrize("policy,bits", [("fixed", 4), ("fixed", 8), ("fixed", 16), ("fp32", 0)])
def test_inner_product_search(ipctx, policy, bits):
    g = _gpu(ipctx, 10, 6, policy=policy, bits=bits)
    check_coarse(g["coarse"], ipctx["idx"], ipctx["Q"])
    certify_probes(g["probes"], ipctx["idx"], ipctx["Q"], 6)
    ref = _oracle(ipctx, 10, 6, g, policy=policy, bits=bits)
    if policy == "fp32":
        compare_fp32(g, ref, ipctx["idx"], ipctx["Q"])
    else:
        compare_integer(g, ref)


@pytest.fixture(scope="module")
def e4ctx():
    # anisotropic clusters on the e4m3 operand grid, d/M = 8 (the high-dim shape)
    return _small("aniso", grid_kind="e4m3", d=96, M=12, nlist=24)


@pytest.mark.parametrize("dtype", [amp.AMP_LUT_BF16, amp.AMP_LUT_F16])
@pytest.mark.parametrize("bits", [4, 8, 16])
def test_lut_build_dtypes_are_bit_exact_on_the_e4m3_grid(e4ctx, dtype, bits):
    g = _gpu(e4ctx, 20, 5, policy="fixed", bits=bits, lut_dtype=dtype)
    certify_probes(g["probes"], e4ctx["idx"], e4ctx["Q"], 5)
    ref = _oracle(e4ctx, 20, 5, g, policy="fixed", bits=bits)
    compare_integer(g, ref)


@pytest.mark.parametrize("M,d", [(4, 16), (32, 128), (40, 80), (64, 128), (128, 256)])
def test_subspace_counts(M, d):
    """Subspace counts without a specialised scan variant (4, 40: the generic
    kernel, one LUT word per row) and with one (32: two-word rows; 64; 128:
    512-thread workgroups), including d/M = 2 and 4."""
    ctx = _small("aniso", d=d, M=M, nlist=16, n=6000, n_comp=24, nq=24, seed=31 + M)
    for policy, bits in (("fixed", 4), ("fixed", 16), ("fp32", 0)):
        g = _gpu(ctx, 10, 4, policy=policy, bits=bits)
        certify_probes(g["probes"], ctx["idx"], ctx["Q"], 4)
        ref = _oracle(ctx, 10, 4, g, policy=policy, bits=bits)
        if policy == "fp32":
            compare_fp32(g, ref, ctx["idx"], ctx["Q"])
        else:
            compare_integer(g, ref)


@pytest.mark.parametrize("bits", [4, 12])
def test_fp16_lut_build_on_the_9bit_grid(tiny, bits):
    g = _gpu(tiny, 10, 8, policy="fixed", bits=bits, lut_dtype=amp.AMP_LUT_F16)
    ref = _oracle(tiny, 10, 8, g, policy="fixed", bits=bits)
    compare_integer(g, ref)


def test_fp8_build_needs_the_e4m3_grid(tiny, e4ctx):
    # the FP8 build is offered on the e4m3 operand grid only (the 9-bit grid's
    # integers are not all e4m3 values)
    with pytest.raises(amp.AmpError) as e:
        amp.amp_search(tiny["h"], tiny["Q"][:2], 5, 2, policy="fixed", bits=8, lut_dtype=amp.AMP_LUT_F8E4M3)
    assert e.value.status == amp.AMP_EINVAL
    with pytest.raises(amp.AmpError) as e:
        amp.amp_search(tiny["h"], tiny["Q"][:2], 5, 2, policy="fixed", bits=8, lut_dtype=7)
    assert e.value.status == amp.AMP_EINVAL
    amp.amp_search(e4ctx["h"], e4ctx["Q"][:2], 5, 2, policy="fixed", bits=8, lut_dtype=amp.AMP_LUT_F8E4M3)


def _export_search(torch, ctx, k, nprobe, want_t=True, **pol):
    """Device-mode search with the LUT export; returns numpy arrays."""
    Q = ctx["Q"]
    nq, M = len(Q), ctx["idx"]["M"]
    npmax = int(np.max(nprobe))
    kmax = int(np.max(k))
    dev = "cuda"
    o = dict(ids=torch.empty((nq, kmax), dtype=torch.int64, device=dev),
             dist=torch.empty((nq, kmax), dtype=torch.float32, device=dev),
             qdist=torch.empty((nq, kmax), dtype=torch.int64, device=dev),
             probes=torch.empty((nq, npmax), dtype=torch.int32, device=dev),
             bits=torch.empty((nq, npmax), dtype=torch.uint8, device=dev),
             status=torch.zeros(1, dtype=torch.int32, device=dev),
             lut_q=torch.zeros((nq, npmax, M, 256), dtype=torch.int16, device=dev),
             lut_shift=torch.zeros((nq, npmax), dtype=torch.int32, device=dev),
             lut_base=torch.zeros((nq, npmax), dtype=torch.int64, device=dev))
    if want_t:
        o["lut_t"] = torch.zeros((nq, npmax, M, 256), dtype=torch.int32, device=dev)
    s = torch.cuda.Stream()
    amp.amp_search(ctx["h"], torch.from_numpy(Q).to(dev), k, nprobe, out=o, stream=s, **pol)
    s.synchronize()
    out = {kk: v.cpu().numpy() for kk, v in o.items()}
    out["lut_q"] = out["lut_q"].view(np.uint16)
    return out


def _replay(ctx, g, k):
    """The oracle's integer DC and TS stages on the GPU's exported LUTs:
    must reproduce the GPU's ids and integer distances exactly."""
    idx = ctx["idx"]
    for i in range(len(ctx["Q"])):
        P = g["probes"][i]
        P = P[P >= 0]
        tables = [(g["lut_q"][i, r], int(g["lut_shift"][i, r]), int(g["lut_base"][i, r])) for r in range(len(P))]
        kk = int(np.broadcast_to(k, (len(ctx["Q"]),))[i])
        ids, qd = oracle.dc_ts(idx, P, tables, kk)
        assert np.array_equal(g["ids"][i, :kk], ids), i
        assert np.array_equal(g["qdist"][i, :kk], qd), i


@pytest.mark.parametrize("dtype", [amp.AMP_LUT_BF16, amp.AMP_LUT_F8E4M3])
def test_lut_export_replays_exactly_and_bf16_export_is_the_oracles(highdim_shape, dtype):
    """Replay invariant: the oracle's integer DC and TS stages applied to the
    exported per-pair (Q, s, base) reproduce the GPU's ids and integer
    distances, for the exact BF16 build and for the FP8 build (high-dim
    shape: d 960, PQ120, e4m3 grid, k 100).  The BF16 export equals the
    oracle's own quantised LUTs.  The FP8 MFMA's dot products of e4m3
    integers are not always exact (about 0.5% of the entries of this shape
    are off by 2 or 4 out of up to 5.6e5); the FP8 entries before
    quantisation must stay within 16 of the exact integer LUT."""
    torch = pytest.importorskip("torch")
    ctx, w = highdim_shape
    m = _spread_model(ctx, 12)
    amp.amp_index_set_predictor(ctx["h"], m)
    idx = ctx["idx"]
    cbi, _ = oracle.index_grid(idx)
    inv = 2.0 ** -idx["grid_e"]
    for policy, bits, kw in (("fixed", 4, {}), ("fixed", 16, {}), ("adaptive", 0, dict(allowed=(4, 8, 16)))):
        g = _export_search(torch, ctx, 100, 12, policy=policy, bits=bits, lut_dtype=dtype, **kw)
        assert int(g["status"][0]) == amp.AMP_OK
        _replay(ctx, g, 100)
        worst = 0.0
        for i in range(0, len(ctx["Q"]), 3):
            for r in range(12):
                p = int(g["probes"][i, r])
                ri = oracle.grid(oracle.residual_f32(ctx["Q"][i], idx["centroids"][p]).astype(np.float64) * inv,
                                 idx["grid_kind"])
                T = oracle.lut_int(ri, cbi, "l2")
                Tg = g["lut_t"][i, r].astype(np.int64)
                if dtype == amp.AMP_LUT_BF16:
                    assert np.array_equal(Tg, T)
                    Qt, sh, base = oracle.quantize_lut(T, int(g["bits"][i, r]))
                    assert int(g["lut_shift"][i, r]) == sh and int(g["lut_base"][i, r]) == base
                    assert np.array_equal(g["lut_q"][i, r].astype(np.int64), Qt)
                else:
                    worst = max(worst, float(np.abs(Tg - T).max()))
        if dtype == amp.AMP_LUT_F8E4M3:
            print(f"fp8 {policy}{bits}: max |T_fp8 - T| = {worst:.0f}")
            assert worst <= 16


def test_fp8_inner_product_build_replays_exactly():
    # inner product on the e4m3 grid: the queries' tables on the FP8 MFMA
    torch = pytest.importorskip("torch")
    ctx = _small("vmf", metric="ip", grid_kind="e4m3", d=64, M=8, nlist=24, nq=24)
    for bits in (4, 8, 16):
        g = _export_search(torch, ctx, 10, 6, want_t=False, policy="fixed", bits=bits, lut_dtype=amp.AMP_LUT_F8E4M3)
        _replay(ctx, g, 10)
        gb = _export_search(torch, ctx, 10, 6, want_t=False, policy="fixed", bits=bits, lut_dtype=amp.AMP_LUT_BF16)
        _replay(ctx, gb, 10)
        ref = _oracle(ctx, 10, 6, gb, policy="fixed", bits=bits)
        compare_integer(dict(ids=gb["ids"], qdist=gb["qdist"], dist=gb["dist"]), ref)


def test_graph_replay_matches_eager(tiny):
    """A captured search replayed several times, with other eager work and
    synchronisations between replays and new query contents before some of
    them, gives the eager result every time."""
    torch = pytest.importorskip("torch")
    Q = tiny["Q"]
    nq = len(Q)
    s = torch.cuda.Stream()
    qd = torch.from_numpy(Q).cuda()

    def outs():
        return dict(ids=torch.empty((nq, 10), dtype=torch.int64, device="cuda"),
                    dist=torch.empty((nq, 10), dtype=torch.float32, device="cuda"),
                    qdist=torch.empty((nq, 10), dtype=torch.int64, device="cuda"),
                    bits=torch.empty((nq, 8), dtype=torch.uint8, device="cuda"))

    Q2 = np.ascontiguousarray(Q[::-1])
    want = {0: amp.amp_search(tiny["h"], Q, 10, 8, policy="fixed", bits=8),
            1: amp.amp_search(tiny["h"], Q2, 10, 8, policy="fixed", bits=8)}
    og = outs()
    for rep in range(5):
        src = rep % 2
        with torch.cuda.stream(s):
            qd.copy_(torch.from_numpy(Q if src == 0 else Q2).cuda())
            for v in og.values():
                v.fill_(-1)
        amp.amp_search(tiny["h"], qd, 10, 8, policy="fixed", bits=8, out=og, stream=s, graph=True)
        s.synchronize()
        # unrelated eager work between replays
        x = torch.randn(512, 512, device="cuda")
        (x @ x).sum().item()
        torch.cuda.synchronize()
        assert np.array_equal(og["ids"].cpu().numpy(), want[src]["ids"]), rep
        assert np.array_equal(og["qdist"].cpu().numpy(), want[src]["qdist"]), rep
        assert np.array_equal(og["dist"].cpu().numpy().view(np.uint32), want[src]["dist"].view(np.uint32)), rep
        assert np.all(og["bits"].cpu().numpy() == 8)
    # an eager device-mode search on the same index afterwards is unaffected
    oe = outs()
    amp.amp_search(tiny["h"], qd, 10, 8, policy="fixed", bits=8, out=oe, stream=s)
    s.synchronize()
    assert np.array_equal(oe["ids"].cpu().numpy(), og["ids"].cpu().numpy())


def test_graph_mode_rejections(tiny):
    torch = pytest.importorskip("torch")
    Q = tiny["Q"][:4]
    qd = torch.from_numpy(Q).cuda()
    o = dict(ids=torch.empty((4, 10), dtype=torch.int64, device="cuda"),
             dist=torch.empty((4, 10), dtype=torch.float32, device="cuda"))
    s = torch.cuda.Stream()
    bad = [dict(stream=None),                                    # null stream
           dict(stream=s, stage_ms=True),
           dict(stream=s, policy="explicit", explicit_bits=np.full((4, 8), 8, np.uint8))]
    for kw in bad:
        args = dict(policy="fixed", bits=8)
        args.update(kw)
        with pytest.raises(amp.AmpError) as e:
            amp.amp_search(tiny["h"], qd, 10, 8, out=o, graph=True, **args)
        assert e.value.status == amp.AMP_EINVAL
    with pytest.raises(amp.AmpError):
        amp.amp_search(tiny["h"], qd, [10, 5, 10, 5], 8, out=o, stream=s, graph=True)
    with pytest.raises(amp.AmpError):
        amp.amp_search(tiny["h"], Q, 10, 8, graph=True)


# ---- the other workload shapes at sizes the oracle finishes in seconds
def _shape(name, n, nq, nlist, nprobe, seed_off=0):
    import dataclasses
    w = dataclasses.replace(WORKLOADS[name], n=n, nq=nq, nlist=nlist, nprobe=nprobe)
    base = make_base(w)
    idx = build_index(base, w.nlist, w.M, iters=8, seed=w.seed + seed_off, integer_data=w.integer_data,
                      grid_kind=w.grid_kind, metric=w.metric)
    return _ctx(idx, make_queries(w, nq), base), w


@pytest.fixture(scope="module")
def skewed_shape():
    # d 96, PQ24 (the M = 24 register variant), Zipf-skewed lists, uneven nprobe
    return _shape("skewed", 60_000, 48, 256, 64)


def test_skewed_shape_uneven_nprobe(skewed_shape):
    ctx, w = skewed_shape
    sizes = ctx["idx"]["list_sizes"]
    assert sizes.max() >= 4 * np.median(sizes)  # Zipf-skewed list sizes
    npq = np.random.default_rng(3).integers(8, 65, size=len(ctx["Q"])).astype(np.int32)
    m = _spread_model(ctx, 64)
    amp.amp_index_set_predictor(ctx["h"], m)
    for policy, bits in (("fixed", 4), ("fixed", 16), ("adaptive", 0), ("fp32", 0)):
        g = _gpu(ctx, 10, npq, policy=policy, bits=bits)
        certify_probes(g["probes"], ctx["idx"], ctx["Q"], npq)
        kw = dict(model=m) if policy == "adaptive" else {}
        ref = _oracle(ctx, 10, npq, g, policy=policy, bits=bits, **kw)
        if policy == "fp32":
            compare_fp32(g, ref, ctx["idx"], ctx["Q"])
        else:
            compare_integer(g, ref)
            if policy == "adaptive":
                assert np.array_equal(g["bits"], ref["bits"])


@pytest.fixture(scope="module")
def highdim_shape():
    # d 960, PQ120 (d/M = 8) on the e4m3 grid, k 100 (more than a wave holds: every
    # lane minimum of a pair goes to the phase-1 bound buffer)
    return _shape("highdim", 16_000, 12, 32, 12)


@pytest.mark.parametrize("dtype", [amp.AMP_LUT_BF16, amp.AMP_LUT_F16])
def test_highdim_shape_k100(highdim_shape, dtype):
    ctx, w = highdim_shape
    m = _spread_model(ctx, 12)
    amp.amp_index_set_predictor(ctx["h"], m)
    for policy, bits in (("fixed", 4), ("fixed", 16), ("adaptive", 0), ("fp32", 0)):
        if policy == "fp32" and dtype != amp.AMP_LUT_BF16:
            continue
        kw = dict(allowed=(4, 8, 16)) if policy == "adaptive" else {}
        g = _gpu(ctx, 100, 12, policy=policy, bits=bits, lut_dtype=dtype, **kw)
        certify_probes(g["probes"], ctx["idx"], ctx["Q"], 12)
        if policy == "adaptive":
            kw["model"] = m
        ref = _oracle(ctx, 100, 12, g, policy=policy, bits=bits, **kw)
        if policy == "fp32":
            compare_fp32(g, ref, ctx["idx"], ctx["Q"])
        else:
            compare_integer(g, ref)
            assert np.array_equal(g["bits"], ref["bits"])


@pytest.fixture(scope="module")
def serving_shape():
    # d 768 unit-normalised, inner product, PQ96 (generic variant)
    return _shape("serving", 20_000, 24, 32, 16)


def test_serving_shape_inner_product_mixed_k(serving_shape):
    ctx, w = serving_shape
    r = np.random.default_rng(11)
    kq = r.choice([10, 50, 100], size=len(ctx["Q"])).astype(np.int32)
    npq = r.choice([4, 8, 16], size=len(ctx["Q"])).astype(np.int32)
    for policy, bits in (("fixed", 4), ("fixed", 8), ("fixed", 16), ("fp32", 0)):
        g = _gpu(ctx, kq, npq, policy=policy, bits=bits)
        certify_probes(g["probes"], ctx["idx"], ctx["Q"], npq)
        ref = _oracle(ctx, kq, npq, g, policy=policy, bits=bits)
        if policy == "fp32":
            compare_fp32(g, ref, ctx["idx"], ctx["Q"])
        else:
            compare_integer(g, ref)


def test_device_queries_must_be_16_byte_aligned(tiny):
    torch = pytest.importorskip("torch")
    Q = tiny["Q"][:5]
    flat = torch.from_numpy(np.ascontiguousarray(Q).ravel()).cuda()
    o = dict(ids=torch.empty((4, 5), dtype=torch.int64, device="cuda"),
             dist=torch.empty((4, 5), dtype=torch.float32, device="cuda"))
    bad = flat[1:1 + 4 * Q.shape[1]].view(4, Q.shape[1])  # 4-byte offset
    with pytest.raises(amp.AmpError) as e:
        amp.amp_search(tiny["h"], bad, 5, 4, out=o, stream=torch.cuda.current_stream())
    assert e.value.status == amp.AMP_EINVAL
    good = flat[Q.shape[1]:].view(4, Q.shape[1])  # one row in: aligned (d % 4 == 0)
    amp.amp_search(tiny["h"], good, 5, 4, out=o, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    ref = amp.amp_search(tiny["h"], Q[1:], 5, 4)
    assert np.array_equal(o["ids"].cpu().numpy(), ref["ids"])


@pytest.mark.parametrize("nlist,nprobe", [(64, 5), (1000, 37), (256, 100), (1500, 8), (2048, 64), (3000, 130),
                                          (4096, 256), (5000, 20)])
def test_probe_ties_follow_list_ids(nlist, nprobe):
    """Duplicated centroids give bit-identical coarse distances: the probe
    order must then follow the list id, including at the nprobe boundary
    (wave-level selection for nlist <= 1024 and nprobe <= 64, workgroup-level
    selection for nlist <= 4096, a sort of the whole row beyond)."""
    r = np.random.default_rng(nlist + nprobe)
    M, dsub = 8, 4
    d = M * dsub
    C = r.integers(-20, 21, size=(nlist, d)).astype(np.float32)
    dup = r.choice(nlist, size=min(nlist, 3 * nprobe), replace=False)
    C[dup] = C[dup[0]]  # one point repeated many times
    n_per = 2
    idx = dict(d=d, M=M, dsub=dsub, nlist=nlist, ksub=256, metric="l2", grid_kind="u9", grid_e=0,
               centroids=C, codebook=r.integers(-3, 4, size=(M, 256, dsub)).astype(np.float32),
               list_offsets=np.arange(0, nlist * n_per + 1, n_per), ids=np.arange(nlist * n_per, dtype=np.int64),
               codes=r.integers(0, 256, size=(nlist * n_per, M)).astype(np.uint8),
               list_sizes=np.full(nlist, n_per, np.int32), radq=np.full(nlist, 10, np.int32))
    Q = np.repeat(C[dup[:1]], 6, axis=0) + r.integers(-1, 2, size=(6, d)).astype(np.float32)
    ctx = _ctx(idx, Q)
    g = _gpu(ctx, 3, nprobe, policy="fixed", bits=16)
    for i, q in enumerate(Q):
        want = oracle.select_probes(oracle.coarse_distances(q, C), nprobe)
        assert np.array_equal(g["probes"][i], want), (i, g["probes"][i], want)


def test_bf16_queries_search_as_their_fp32_values(tiny):
    torch = pytest.importorskip("torch")
    from _parity import bf16_bits, bf16_widen
    Qb = bf16_bits(tiny["Q"])
    Qw = bf16_widen(Qb)
    g = amp.amp_search(tiny["h"], Qb, 10, 8, policy="fixed", bits=8, want_probes=True)
    ref = oracle.search(tiny["idx"], Qw, 10, 8, probes=g["probes"], policy="fixed", bits=8)
    certify_probes(g["probes"], tiny["idx"], Qw, 8)
    compare_integer(g, ref)
    w = amp.amp_search(tiny["h"], Qw, 10, 8, policy="fixed", bits=8)
    assert np.array_equal(w["ids"], g["ids"]) and np.array_equal(w["qdist"], g["qdist"])
    # device mode from a torch bfloat16 tensor
    qd = torch.from_numpy(Qw).cuda().to(torch.bfloat16)
    out = dict(ids=torch.empty((len(Qw), 10), dtype=torch.int64, device="cuda"),
               dist=torch.empty((len(Qw), 10), dtype=torch.float32, device="cuda"),
               qdist=torch.empty((len(Qw), 10), dtype=torch.int64, device="cuda"))
    amp.amp_search(tiny["h"], qd, 10, 8, policy="fixed", bits=8, out=out, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert np.array_equal(out["ids"].cpu().numpy(), g["ids"])
    assert np.array_equal(out["qdist"].cpu().numpy(), g["qdist"])
    fp = amp.amp_search(tiny["h"], Qb, 10, 8, policy="fp32")
    fw = amp.amp_search(tiny["h"], Qw, 10, 8, policy="fp32")
    assert np.array_equal(fp["ids"], fw["ids"]) and np.array_equal(fp["dist"].view(np.uint32), fw["dist"].view(np.uint32))


def test_device_mode_per_query_arrays_may_be_reused_at_return(tiny):
    torch = pytest.importorskip("torch")
    Q = tiny["Q"]
    r = np.random.default_rng(8)
    qd = torch.from_numpy(Q).cuda()
    s = torch.cuda.Stream()
    outs, want = [], []
    kk = np.empty(len(Q), np.int32)
    npb = np.empty(len(Q), np.int32)
    with torch.cuda.stream(s):
        for rep in range(4):
            kk[:] = r.integers(1, 11, len(Q))
            npb[:] = r.integers(1, 9, len(Q))
            want.append(amp.amp_search(tiny["h"], Q, kk.copy(), npb.copy(), policy="fixed", bits=12))
            o = dict(ids=torch.empty((len(Q), 10), dtype=torch.int64, device="cuda"),
                     dist=torch.empty((len(Q), 10), dtype=torch.float32, device="cuda"),
                     qdist=torch.empty((len(Q), 10), dtype=torch.int64, device="cuda"))
            amp.amp_search(tiny["h"], qd, kk, npb, policy="fixed", bits=12, out=o, stream=s)
            outs.append((o, int(kk.max())))
            kk[:] = 1  # overwritten as soon as the call returns
            npb[:] = 1
    s.synchronize()
    for (o, km), w in zip(outs, want):
        assert np.array_equal(o["ids"].cpu().numpy()[:, :km], w["ids"])
        assert np.array_equal(o["qdist"].cpu().numpy()[:, :km], w["qdist"])


@pytest.mark.parametrize("policy,bits", [("fixed", 16), ("fixed", 4), ("fp32", 0)])
def test_bound_spans_probes_when_the_nearest_list_is_smaller_than_k(monkeypatch, policy, bits):
    # lists of ~25 vectors, k = 50: the phase-1 bound must combine several
    # nearest lists; a small candidate buffer shows a missing bound as an
    # overflow
    c = _small("vmf", metric="ip", n=6_000, d=64, n_comp=64, nlist=256, M=16, seed=21, nq=24)
    monkeypatch.setenv("AMP_CAPQ", "512")
    g = _gpu(c, 50, 64, policy=policy, bits=bits)
    ref = _oracle(c, 50, 64, g, policy=policy, bits=bits)
    if policy == "fp32":
        compare_fp32(g, ref, c["idx"], c["Q"])
    else:
        compare_integer(g, ref)


@pytest.mark.parametrize("k,nprobe", [(65, 8), (200, 8), (300, 8), (700, 1)])
def test_top_k_select_and_sort_paths(tiny, k, nprobe):
    # the phase-1 bound and the merge take the k-th smallest key by radix
    # select (4-bit LUTs: many equal keys); the merge ranks the candidates up
    # to it when there are at most 256 (k = 65, 200) and sorts them all when
    # there are more (k = 300) or when a query has at most k candidates (one
    # probed list of about 300 vectors, k = 700: rows padded with -1)
    g = _gpu(tiny, k, nprobe, policy="fixed", bits=4)
    ref = _oracle(tiny, k, nprobe, g, policy="fixed", bits=4)
    compare_integer(g, ref)
    if k == 700:
        sizes = np.diff(tiny["idx"]["list_offsets"])[g["probes"][:, 0]]
        assert (sizes < k).any()
        assert (g["ids"][sizes < k, -1] == -1).all()


@pytest.mark.parametrize("policy,bits", [("fixed", 4), ("fixed", 16), ("fp32", 0)])
def test_candidate_overflow_is_resolved_by_rerunning_phase_two(tiny, monkeypatch, capfd, policy, bits):
    # a 64-entry candidate buffer for k = 10: queries whose candidates under
    # the phase-1 bound overflow it (4-bit LUTs: about 120 per query, with
    # many ties) are re-scanned with a tighter (distance, id) bound
    monkeypatch.setenv("AMP_CAPQ", "64")
    monkeypatch.setenv("AMP_STATS", "1")
    g = _gpu(tiny, 10, 8, policy=policy, bits=bits)
    err = capfd.readouterr().err
    ref = _oracle(tiny, 10, 8, g, policy=policy, bits=bits)
    if policy == "fp32":
        compare_fp32(g, ref, tiny["idx"], tiny["Q"])
    else:
        compare_integer(g, ref)
    if policy == "fixed" and bits == 4:
        assert "phase-2 re-runs: 1" in err, err


@pytest.mark.parametrize("policy,bits", [("fixed", 8), ("fp32", 0), ("adaptive", 0)])
def test_work_counters_account_for_every_pair(tiny, policy, bits):
    if policy == "adaptive":
        amp.amp_index_set_predictor(tiny["h"], _spread_model(tiny, 8))
    g = amp.amp_search(tiny["h"], tiny["Q"], 10, 8, policy=policy, bits=bits, want_probes=True, work=True)
    wk = g["work"]
    P = g["probes"]
    sizes = np.diff(tiny["idx"]["list_offsets"])
    assert wk["live_pairs"] + wk["dead_pairs"] == (P >= 0).sum()
    assert 0 < wk["scan_bytes"] <= sizes[P[P >= 0]].sum() * tiny["idx"]["M"]
    # pairs skipped whole scan nothing: the bytes are those of the live pairs' lists
    assert wk["live_pairs"] > 0
    # the units read each chunk's codes once (at most the pairs' code bytes)
    # plus their LUT sources (at most a table or the residual rows per pair
    # and the codebook per unit)
    ix = tiny["idx"]
    d, M = ix["d"], ix["M"]
    n = int((P >= 0).sum())
    lut_src = n * max(M * 256 * 4, d * 4) + n * (d * 4 + M * 256 * ix["dsub"] * 4)
    assert 0 < wk["unit_bytes"] <= wk["scan_bytes"] + lut_src


@pytest.fixture(scope="module")
def l1ctx():
    # the L1 mode of the distance module: same index construction, L1 search
    return _small("iso", metric="l1", n=12_000, d=64, n_comp=48, nlist=32, M=16, seed=31, nq=40)


def _l1_probes_ok(g, ctx, nprobe):
    C = np.asarray(ctx["idx"]["centroids"], np.float32)
    for i, q in enumerate(ctx["Q"]):
        D64 = oracle.coarse_distances(q, C, "l1")
        assert np.allclose(g["coarse"][i], D64, rtol=1e-5, atol=1e-5 * np.abs(D64).max())
        want = oracle.select_probes(D64, nprobe)
        for a, b in zip(g["probes"][i][:nprobe].tolist(), want.tolist()):
            if a != b:  # only FP32 near-ties may swap
                assert abs(D64[a] - D64[b]) <= 1e-5 * D64.max(), (i, a, b)


@pytest.mark.parametrize("policy,bits", [("fixed", 4), ("fixed", 8), ("fixed", 16), ("fp32", 0)])
def test_l1_search(l1ctx, policy, bits):
    g = _gpu(l1ctx, 10, 6, policy=policy, bits=bits)
    _l1_probes_ok(g, l1ctx, 6)
    ref = _oracle(l1ctx, 10, 6, g, policy=policy, bits=bits)
    if policy == "fp32":
        compare_fp32(g, ref, l1ctx["idx"], l1ctx["Q"])
    else:
        compare_integer(g, ref)


def test_l1_adaptive_search(l1ctx):
    m = _spread_model(l1ctx, 6)
    amp.amp_index_set_predictor(l1ctx["h"], m)
    g = _gpu(l1ctx, 10, 6, policy="adaptive")
    ref = _oracle(l1ctx, 10, 6, g, policy="adaptive", model=m)
    assert np.array_equal(g["bits"], ref["bits"])
    compare_integer(g, ref)


# ---- nprobe above 64 end to end, the one-word-row scan variants, device-side
# ---- status and device-resident per-query sizes
def test_skewed_shape_nprobe_up_to_128(skewed_shape):
    # per-query nprobe U[8, 128]: the workgroup top-nprobe, 128 pair slots per
    # query in the predictor, the queue at that width
    ctx, w = skewed_shape
    npq = np.random.default_rng(4).integers(8, 129, size=len(ctx["Q"])).astype(np.int32)
    assert npq.max() > 64
    m = _spread_model(ctx, 128, seed=1)
    amp.amp_index_set_predictor(ctx["h"], m)
    for policy, bits in (("fixed", 4), ("fixed", 16), ("adaptive", 0), ("fp32", 0)):
        g = _gpu(ctx, 10, npq, policy=policy, bits=bits)
        certify_probes(g["probes"], ctx["idx"], ctx["Q"], npq)
        kw = dict(model=m) if policy == "adaptive" else {}
        ref = _oracle(ctx, 10, npq, g, policy=policy, bits=bits, **kw)
        if policy == "fp32":
            compare_fp32(g, ref, ctx["idx"], ctx["Q"])
        else:
            compare_integer(g, ref)
            if policy == "adaptive":
                assert np.array_equal(g["bits"], ref["bits"])


@pytest.fixture(scope="module")
def serving_wide():
    # the serving shape with enough lists for nprobe 256 (d 768, inner product, PQ96)
    return _shape("serving", 40_000, 12, 512, 256)


def test_serving_shape_nprobe_256_k100(serving_wide):
    ctx, w = serving_wide
    r = np.random.default_rng(12)
    nq = len(ctx["Q"])
    kq = r.choice([10, 50, 100], size=nq).astype(np.int32)
    npq = r.choice([16, 64, 256], size=nq).astype(np.int32)
    kq[0], npq[0] = 100, 256
    m = _spread_model(ctx, 256, seed=2)
    amp.amp_index_set_predictor(ctx["h"], m)
    for policy, bits in (("fixed", 4), ("fixed", 16), ("adaptive", 0), ("fp32", 0)):
        g = _gpu(ctx, kq, npq, policy=policy, bits=bits)
        certify_probes(g["probes"], ctx["idx"], ctx["Q"], npq)
        kw = dict(model=m) if policy == "adaptive" else {}
        ref = _oracle(ctx, kq, npq, g, policy=policy, bits=bits, **kw)
        if policy == "fp32":
            compare_fp32(g, ref, ctx["idx"], ctx["Q"])
        else:
            compare_integer(g, ref)
            if policy == "adaptive":
                assert np.array_equal(g["bits"], ref["bits"])


@pytest.mark.parametrize("shape", ["midint", "skewed_shape"])
def test_one_word_row_variants_match_the_oracle(shape, request, monkeypatch):
    # the M = 16 and M = 24 scan variants with one-word LUT rows (NR = 1, the
    # sparse-batch regime) forced on a few queries
    ctx = request.getfixturevalue(shape)
    if isinstance(ctx, tuple):
        ctx = ctx[0]
    monkeypatch.setenv("AMP_NARROW", "1")
    sub = dict(ctx, Q=np.ascontiguousarray(ctx["Q"][:6]))
    m = _spread_model(sub, 8, seed=3)
    amp.amp_index_set_predictor(ctx["h"], m)
    for policy, bits in (("fixed", 4), ("fixed", 8), ("fixed", 16), ("adaptive", 0), ("fp32", 0)):
        g = _gpu(sub, 10, 8, policy=policy, bits=bits)
        kw = dict(model=m) if policy == "adaptive" else {}
        ref = _oracle(sub, 10, 8, g, policy=policy, bits=bits, **kw)
        if policy == "fp32":
            compare_fp32(g, ref, sub["idx"], sub["Q"])
        else:
            compare_integer(g, ref)


def _dev_out(torch, nq, kmax, npmax=None):
    o = dict(ids=torch.empty((nq, kmax), dtype=torch.int64, device="cuda"),
             dist=torch.empty((nq, kmax), dtype=torch.float32, device="cuda"),
             qdist=torch.empty((nq, kmax), dtype=torch.int64, device="cuda"),
             status=torch.full((1,), 12345, dtype=torch.int32, device="cuda"))
    if npmax:
        o["probes"] = torch.empty((nq, npmax), dtype=torch.int32, device="cuda")
    return o


def test_device_mode_overflow_is_reported_through_the_status_word(tiny, monkeypatch):
    # a 64-entry candidate buffer and no re-runs: the 4-bit searches of these
    # queries overflow it (about 120 candidates each); the device-mode search
    # returns at once and its status word reads AMP_EOVERFLOW; without the
    # overflow it reads AMP_OK
    torch = pytest.importorskip("torch")
    Q = tiny["Q"]
    nq = len(Q)
    qd = torch.from_numpy(Q).cuda()
    s = torch.cuda.Stream()
    o = _dev_out(torch, nq, 10)
    amp.amp_search(tiny["h"], qd, 10, 8, policy="fixed", bits=4, out=o, stream=s)
    s.synchronize()
    assert int(o["status"].item()) == amp.AMP_OK
    monkeypatch.setenv("AMP_CAPQ", "64")
    monkeypatch.setenv("AMP_RERUNS", "0")
    o = _dev_out(torch, nq, 10)
    amp.amp_search(tiny["h"], qd, 10, 8, policy="fixed", bits=4, out=o, stream=s)
    s.synchronize()
    assert int(o["status"].item()) == amp.AMP_EOVERFLOW
    h = amp.amp_search(tiny["h"], Q, 10, 8, policy="fixed", bits=4, want_status=True)
    assert h["status"] == amp.AMP_EOVERFLOW
    # with the re-runs the same buffer suffices, and the status says so
    monkeypatch.setenv("AMP_RERUNS", "2")
    o = _dev_out(torch, nq, 10)
    amp.amp_search(tiny["h"], qd, 10, 8, policy="fixed", bits=4, out=o, stream=s)
    s.synchronize()
    assert int(o["status"].item()) == amp.AMP_OK


def test_graph_replay_with_device_resident_sizes(tiny):
    """Per-query k and nprobe in device memory: one captured graph replayed
    with new sizes (and new queries) gives, every time, the eager search with
    the same sizes as host arrays."""
    torch = pytest.importorskip("torch")
    Q = tiny["Q"]
    nq = len(Q)
    r = np.random.default_rng(21)
    s = torch.cuda.Stream()
    qd = torch.from_numpy(Q).cuda()
    kd = torch.empty(nq, dtype=torch.int32, device="cuda")
    npd = torch.empty(nq, dtype=torch.int32, device="cuda")
    o = _dev_out(torch, nq, 20, 12)
    for rep in range(4):
        ks = r.integers(1, 21, size=nq).astype(np.int32)
        nps = r.integers(1, 13, size=nq).astype(np.int32)
        Qr = Q if rep % 2 == 0 else np.ascontiguousarray(Q[::-1])
        with torch.cuda.stream(s):
            qd.copy_(torch.from_numpy(Qr).cuda())
            kd.copy_(torch.from_numpy(ks).cuda())
            npd.copy_(torch.from_numpy(nps).cuda())
            for v in o.values():
                v.fill_(-1)
        amp.amp_search(tiny["h"], qd, kd, npd, kmax=20, npmax=12, policy="fixed", bits=8, out=o, stream=s,
                       graph=True)
        s.synchronize()
        x = torch.randn(256, 256, device="cuda")
        (x @ x).sum().item()
        torch.cuda.synchronize()
        want = amp.amp_search(tiny["h"], Qr, ks, nps, policy="fixed", bits=8, want_probes=True)
        got = {key: v.cpu().numpy() for key, v in o.items()}
        assert int(got["status"][0]) == amp.AMP_OK
        for i in range(nq):
            k, npb = ks[i], nps[i]
            assert np.array_equal(got["ids"][i, :k], want["ids"][i, :k]), (rep, i)
            assert np.array_equal(got["qdist"][i, :k], want["qdist"][i, :k]), (rep, i)
            assert np.array_equal(got["probes"][i, :npb], want["probes"][i, :npb]), (rep, i)
            assert (got["probes"][i, npb:] == -1).all()
            assert (got["ids"][i, k:] == -1).all()


def test_device_sizes_out_of_range_are_clamped_and_reported(tiny):
    torch = pytest.importorskip("torch")
    Q = tiny["Q"][:8]
    qd = torch.from_numpy(Q).cuda()
    ks = np.array([5, 0, 10, 99, 3, 10, -4, 7], np.int32)
    nps = np.array([4, 8, 0, 8, 50, 2, 8, 8], np.int32)
    o = _dev_out(torch, 8, 10, 8)
    s = torch.cuda.Stream()
    amp.amp_search(tiny["h"], qd, torch.from_numpy(ks).cuda(), torch.from_numpy(nps).cuda(), kmax=10, npmax=8,
                   policy="fixed", bits=16, out=o, stream=s)
    s.synchronize()
    assert int(o["status"].item()) == amp.AMP_EINVAL
    kc, nc = np.clip(ks, 1, 10), np.clip(nps, 1, 8)
    want = amp.amp_search(tiny["h"], Q, kc, nc, policy="fixed", bits=16)
    got = o["ids"].cpu().numpy()
    for i in range(8):
        assert np.array_equal(got[i, :kc[i]], want["ids"][i, :kc[i]]), i


# ------------------------------------------- per-(pair, subspace) entry widths
@pytest.mark.parametrize("policy,bits", [("fixed", 4), ("fixed", 8), ("fixed", 16), ("adaptive", 0)])
def test_subspace_granularity_is_bit_exact(tiny, midint, policy, bits):
    """The quantiser with a width per (pair, subspace) (the pair's lane budget
    shared by its subspaces): ids, integer and float distances bit-exact on
    the tiny and the integer-data shapes."""
    for ctx, nprobe in ((tiny, 8), (midint, 16)):
        kw = {}
        if policy == "adaptive":
            m = _spread_model(ctx, nprobe)
            amp.amp_index_set_predictor(ctx["h"], m)
            kw = dict(model=m)
        g = _gpu(ctx, 10, nprobe, policy=policy, bits=bits, granularity="subspace")
        ref = _oracle(ctx, 10, nprobe, g, policy=policy, bits=bits, granularity="subspace", **kw)
        compare_integer(g, ref)


@pytest.mark.parametrize("name,policy,bits", [("ipctx", "fixed", 4), ("ipctx", "fixed", 8), ("e4ctx", "fixed", 4),
                                              ("l1ctx", "fixed", 4), ("l1ctx", "fixed", 8)])
def test_subspace_granularity_other_metrics(request, name, policy, bits):
    ctx = request.getfixturevalue(name)
    nprobe = 6
    g = _gpu(ctx, 10, nprobe, policy=policy, bits=bits, granularity="subspace")
    ref = _oracle(ctx, 10, nprobe, g, policy=policy, bits=bits, granularity="subspace")
    compare_integer(g, ref)


@pytest.mark.parametrize("dtype", [amp.AMP_LUT_BF16, amp.AMP_LUT_F8E4M3])
def test_subspace_granularity_export_replays(highdim_shape, dtype):
    """High-dim shape (PQ120, e4m3 grid, k 100): the exported per-pair tables
    replay the search exactly, and the BF16 export equals the oracle's
    per-subspace quantisation of the exact LUT."""
    torch = pytest.importorskip("torch")
    ctx, w = highdim_shape
    idx = ctx["idx"]
    cbi, _ = oracle.index_grid(idx)
    inv = 2.0 ** -idx["grid_e"]
    g = _export_search(torch, ctx, 100, 12, policy="fixed", bits=4, lut_dtype=dtype, granularity="subspace")
    assert int(g["status"][0]) == amp.AMP_OK
    _replay(ctx, g, 100)
    if dtype == amp.AMP_LUT_BF16:
        for i in range(0, len(ctx["Q"]), 4):
            for r in range(12):
                p = int(g["probes"][i, r])
                ri = oracle.grid(oracle.residual_f32(ctx["Q"][i], idx["centroids"][p]).astype(np.float64) * inv,
                                 idx["grid_kind"])
                Qt, sh, base = oracle.quantize_lut(oracle.lut_int(ri, cbi, "l2"), 4, "subspace")
                assert int(g["lut_shift"][i, r]) == sh and int(g["lut_base"][i, r]) == base
                assert np.array_equal(g["lut_q"][i, r].astype(np.int64), Qt)


@pytest.mark.parametrize("name,policy,bits", [("midint", "fixed", 4), ("midint", "adaptive", 0),
                                              ("ipctx", "fixed", 8), ("tiny", "fp32", 0)])
def test_scanning_every_pair_gives_the_same_results(request, monkeypatch, name, policy, bits):
    """AMP_PAIR_SKIP=0 (a measurement switch) scans the pairs whose base
    exceeds their query's bound too: identical results, more live pairs."""
    ctx = request.getfixturevalue(name)
    if policy == "adaptive":
        amp.amp_index_set_predictor(ctx["h"], _spread_model(ctx, 16))
    g = amp.amp_search(ctx["h"], ctx["Q"], 10, 16 if name == "midint" else 6, policy=policy, bits=bits, work=True)
    monkeypatch.setenv("AMP_PAIR_SKIP", "0")
    g0 = amp.amp_search(ctx["h"], ctx["Q"], 10, 16 if name == "midint" else 6, policy=policy, bits=bits, work=True)
    assert np.array_equal(g["ids"], g0["ids"])
    assert np.array_equal(g["dist"].view(np.uint32), g0["dist"].view(np.uint32))
    assert g0["work"]["dead_pairs"] == 0
    assert g0["work"]["live_pairs"] >= g["work"]["live_pairs"]
