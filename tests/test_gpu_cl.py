"""GPU parity of cluster locating on 8-bit codes with fixed and adaptive
operand widths (oracle/cl.py): per-(slice, sub-space) widths, integer coarse
distances and probes bit-exact, then whole searches from those probes."""
import numpy as np
import pytest

import oracle
import paper_2606_07156_amd as amp
from amp_data import build_index
from amp_data.synth import WORKLOADS, Workload, make_base, make_queries
from oracle import cl as ocl
from _parity import compare_integer

pytestmark = pytest.mark.gpu


def _ctx(w, nlist, M, S, P, nq, metric="l2", integer_data=False, train_nprobe=8, low=4):
    base = make_base(w)
    idx = build_index(base, nlist, M, iters=6, seed=w.seed, integer_data=integer_data, metric=metric)
    h = amp.amp_index_from_arrays(idx)
    amp.amp_index_build_cl_map(h, S, P, iters=10, seed=2)
    rep = amp.amp_index_train_cl_predictor(h, make_queries(w, 40, train=True), train_nprobe, low=low,
                                           n_samples=500)
    amp.amp_index_to_device(h, 0)
    return dict(idx=idx, h=h, Q=make_queries(w, nq), map=amp.amp_index_get_cl_map(h),
                model=amp.amp_index_get_cl_predictor(h), rep=rep)


@pytest.fixture(scope="module")
def clmid():
    # the mid workload's shape (d 128, PQ16, integer data): 16 slices of 8
    # dimensions; 200 lists and 70 queries leave ragged 64 x 64 tiles
    w = WORKLOADS["mid"].scaled(n=50_000, nlist=200)
    return _ctx(w, 200, 16, 16, 40, 70, integer_data=True)


@pytest.fixture(scope="module")
def clip768():
    # inner product, d 768 (the serving shape's dimension): slices of 48
    # dimensions (64-byte MFMA K)
    w = Workload("t", 12_000, 768, 64, 20, 80, 96, 8, 10, "vmf", 31, metric="ip")
    return _ctx(w, 80, 96, 16, 30, 20, metric="ip")


@pytest.fixture(scope="module")
def clskew():
    # d 96 in 16 slices of 6, 100 sub-spaces per slice (two 64-lane groups,
    # four mask words), Zipf-skewed lists
    w = WORKLOADS["skewed"].scaled(n=40_000, nlist=256)
    return _ctx(w, 256, 24, 16, 100, 33)


def _cl(ctx, policy, bits=8, low=4):
    return dict(map=ctx["map"], policy=policy, bits=bits, low=low, model=ctx["model"])


def _check_cl(ctx, g, policy, bits=8, low=4, nprobe=8):
    idx, m = ctx["idx"], ctx["map"]
    for i, q in enumerate(ctx["Q"]):
        P, D, B = ocl.cl_probes(q, idx, m, nprobe, policy, bits, low, ctx["model"])
        assert np.array_equal(g["cl_dist"][i].astype(np.int64), D), (i, policy, bits)
        if "cl_bits" in g:
            assert np.array_equal(g["cl_bits"][i].astype(np.int64), B), (i, low)
        assert np.array_equal(g["probes"][i][:nprobe].astype(np.int64), P), i


@pytest.mark.parametrize("bits", [8, 5, 3])
def test_fixed_width_distances_and_probes(clmid, bits):
    g = amp.amp_search(clmid["h"], clmid["Q"], 10, 8, cl_policy="fixed", cl_bits=bits, want_cl_dist=True,
                       want_probes=True)
    _check_cl(clmid, g, "fixed", bits=bits)


@pytest.mark.parametrize("low,table", [(4, "1"), (4, "0"), (2, "1")])
def test_adaptive_widths_distances_and_probes(clmid, low, table, monkeypatch):
    # table "1": the widths read from the predictor's exact decision table;
    # "0": the regressor evaluated directly (AMP_CL_TABLE=0)
    monkeypatch.setenv("AMP_CL_TABLE", table)
    g = amp.amp_search(clmid["h"], clmid["Q"], 10, 8, cl_policy="adaptive", cl_bits=low, want_cl_dist=True,
                       want_cl_bits=True, want_probes=True)
    _check_cl(clmid, g, "adaptive", low=low)
    share = np.mean([ocl.low_share(b, clmid["map"], low) for b in g["cl_bits"]])
    assert 0 < share < 1


@pytest.mark.parametrize("ctxname", ["clip768", "clskew"])
def test_other_shapes(request, ctxname, monkeypatch):
    ctx = request.getfixturevalue(ctxname)
    for policy, bits, table in (("fixed", 8, "1"), ("fixed", 4, "1"), ("adaptive", 8, "1"), ("adaptive", 8, "0")):
        monkeypatch.setenv("AMP_CL_TABLE", table)
        kw = dict(want_cl_bits=True) if policy == "adaptive" else {}
        g = amp.amp_search(ctx["h"], ctx["Q"], 10, 8, cl_policy=policy, cl_bits=bits if policy == "fixed" else 0,
                           want_cl_dist=True, want_probes=True, **kw)
        _check_cl(ctx, g, policy, bits=bits)


@pytest.mark.parametrize("lut", [("fixed", 8), ("fixed", 16)])
def test_whole_search_from_adaptive_cl(clmid, lut):
    """The rest of the path runs from the integer probes: ids and integer
    distances equal the oracle's search with the same CL policy."""
    policy, bits = lut
    g = amp.amp_search(clmid["h"], clmid["Q"], 10, 8, policy=policy, bits=bits, cl_policy="adaptive",
                       want_probes=True, want_bits=True)
    ref = oracle.search(clmid["idx"], clmid["Q"], 10, 8, policy=policy, bits=bits, cl=_cl(clmid, "adaptive"))
    assert np.array_equal(g["probes"].astype(np.int64), ref["probes"])
    compare_integer(g, ref)


def test_inner_product_whole_search(clip768):
    g = amp.amp_search(clip768["h"], clip768["Q"], 10, 6, policy="fixed", bits=8, cl_policy="adaptive",
                       want_probes=True)
    ref = oracle.search(clip768["idx"], clip768["Q"], 10, 6, policy="fixed", bits=8, cl=_cl(clip768, "adaptive"))
    assert np.array_equal(g["probes"].astype(np.int64), ref["probes"])
    compare_integer(g, ref)


def test_device_mode_graph_replay_matches_host(clmid):
    """Device-resident queries and per-query sizes, captured once and
    replayed: the same probes and results as the host-mode search."""
    torch = pytest.importorskip("torch")
    Q = clmid["Q"]
    nq = len(Q)
    npq = np.random.default_rng(4).integers(4, 13, size=nq).astype(np.int32)
    kq = np.full(nq, 10, np.int32)
    want = amp.amp_search(clmid["h"], Q, kq, npq, policy="fixed", bits=8, cl_policy="adaptive", want_probes=True)
    dev = "cuda"
    o = dict(ids=torch.empty((nq, 10), dtype=torch.int64, device=dev),
             dist=torch.empty((nq, 10), dtype=torch.float32, device=dev),
             qdist=torch.empty((nq, 10), dtype=torch.int64, device=dev),
             probes=torch.empty((nq, 12), dtype=torch.int32, device=dev),
             status=torch.zeros(1, dtype=torch.int32, device=dev),
             cl_dist=torch.empty((nq, 200), dtype=torch.int32, device=dev))
    qd = torch.from_numpy(Q).to(dev)
    kd, nd = torch.from_numpy(kq).to(dev), torch.from_numpy(npq).to(dev)
    s = torch.cuda.Stream()
    for rep in range(3):
        amp.amp_search(clmid["h"], qd, kd, nd, policy="fixed", bits=8, cl_policy="adaptive", out=o, stream=s,
                       graph=True, kmax=10, npmax=12)
        s.synchronize()
        assert int(o["status"][0]) == amp.AMP_OK
        assert np.array_equal(o["ids"].cpu().numpy(), want["ids"]), rep
        assert np.array_equal(o["qdist"].cpu().numpy(), want["qdist"]), rep
        pr = o["probes"].cpu().numpy()
        for i in range(nq):
            assert np.array_equal(pr[i, :npq[i]], want["probes"][i, :npq[i]]), (rep, i)


def test_cl_argument_checks(clmid):
    h, Q = clmid["h"], clmid["Q"]
    with pytest.raises(amp.AmpError):
        amp.amp_search(h, Q, 10, 8, cl_policy="fixed", cl_bits=9)
    with pytest.raises(amp.AmpError):
        amp.amp_search(h, Q, 10, 8, cl_policy="adaptive", cl_bits=8)
    with pytest.raises(amp.AmpError):
        amp.amp_search(h, Q, 10, 8, cl_policy="fixed", cl_bits=8, want_coarse=True)
    with pytest.raises(amp.AmpError):
        amp.amp_search(h, Q, 10, 8, want_cl_dist=True)


def test_max_subspaces_direct_evaluation():
    """P = 1024 sub-spaces per slice (the maximum; the decision table would
    exceed its size cap, so the regressor is evaluated directly): widths,
    distances and probes bit-exact."""
    w = WORKLOADS["mid"].scaled(n=40_000, nlist=1024)
    ctx = _ctx(w, 1024, 16, 16, 1024, 6, integer_data=True)
    g = amp.amp_search(ctx["h"], ctx["Q"], 10, 16, cl_policy="adaptive", want_cl_dist=True, want_cl_bits=True,
                       want_probes=True)
    _check_cl(ctx, g, "adaptive", nprobe=16)
