"""Parity at the benchmark's full size and launch configuration: the mid
workload (1M x 128 integer-valued vectors, IVF1024 / PQ16x256), the whole
10 000-query batch searched in device mode as one captured HIP graph on a
created stream, nprobe 32, k 10, the predictor trained as the benchmark
trains it.  Sampled rows are compared with the oracle one query at a time
(the oracle's result for a query does not depend on the batch); every row is
checked against properties that hold at any size."""
import numpy as np
import pytest

import oracle
import paper_2606_07156_amd as amp
from amp_data.synth import make_queries
from amp_data.workloads import load_or_build
from _parity import certify_probes, check_coarse, compare_fp32, compare_integer

pytestmark = pytest.mark.gpu

# predictor hyper-parameters and training stream of the benchmark
TRAIN_QUERIES, GAMMA, EPSILON, SVR_C, SAMPLES = 256, 10.0, 0.1, 1.0, 1280
ROWS = np.sort(np.random.default_rng(7).choice(10_000, 24, replace=False))


@pytest.fixture(scope="module")
def mid_full():
    pytest.importorskip("torch")
    w, base, idx = load_or_build("mid")
    h = amp.amp_index_from_arrays(idx)
    amp.amp_index_to_device(h, 0)
    amp.amp_index_train_predictor(h, make_queries(w, TRAIN_QUERIES, train=True), w.k, w.nprobe,
                                  gamma=GAMMA, epsilon=EPSILON, C_=SVR_C, n_samples=SAMPLES)
    # list of every base id, for the membership property
    offs = np.asarray(idx["list_offsets"], np.int64)
    list_of = np.empty(w.n, np.int64)
    list_of[np.asarray(idx["ids"], np.int64)] = np.repeat(np.arange(w.nlist), np.diff(offs))
    return dict(w=w, idx=idx, h=h, model=amp.amp_index_get_predictor(h), Q=make_queries(w), list_of=list_of)


def _device_search(ctx, **pol):
    import torch
    w, Q = ctx["w"], ctx["Q"]
    nq, k, npb = len(Q), w.k, w.nprobe
    s = torch.cuda.Stream()
    dev = torch.device("cuda:0")
    qd = torch.from_numpy(Q).to(dev)
    out = dict(ids=torch.empty((nq, k), dtype=torch.int64, device=dev),
               dist=torch.empty((nq, k), dtype=torch.float32, device=dev),
               qdist=torch.empty((nq, k), dtype=torch.int64, device=dev),
               probes=torch.empty((nq, npb), dtype=torch.int32, device=dev),
               bits=torch.empty((nq, npb), dtype=torch.uint8, device=dev),
               coarse=torch.empty((nq, w.nlist), dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    for _ in range(2):  # capture + replay, then one more replay
        amp.amp_search(ctx["h"], qd, k, npb, out=out, stream=s, graph=True, **pol)
    s.synchronize()
    return {key: v.cpu().numpy() for key, v in out.items()}


@pytest.mark.parametrize("policy,bits", [("adaptive", 0), ("fixed", 16), ("fixed", 4), ("fp32", 0)])
def test_full_size_batch(mid_full, policy, bits):
    w, idx, Q = mid_full["w"], mid_full["idx"], mid_full["Q"]
    g = _device_search(mid_full, policy=policy, bits=bits)
    # --- every row: properties of a correct result
    ids, dist = g["ids"], g["dist"]
    assert (ids >= 0).all() and (ids < w.n).all()            # lists hold far more than k vectors
    srt = np.sort(ids, axis=1)
    assert (srt[:, 1:] != srt[:, :-1]).all()                 # no id twice in a row
    assert (np.diff(dist.astype(np.float64), axis=1) >= 0).all()
    member = mid_full["list_of"][ids]                        # every id lies in a probed list
    assert (member[:, :, None] == g["probes"][:, None, :]).any(2).all()
    if policy != "fp32":
        q = g["qdist"]
        assert (np.diff(q, axis=1) >= 0).all()
        # integer data (h = 1): the float distance is the integer one rounded
        assert np.array_equal(dist, q.astype(np.float32))
        assert set(np.unique(g["bits"])) <= ({bits} if policy == "fixed" else {4, 8, 12, 16})
    # --- sampled rows: the oracle, given the GPU's probe sets
    Qs = Q[ROWS]
    check_coarse(g["coarse"][ROWS], idx, Qs)
    certify_probes(g["probes"][ROWS], idx, Qs, w.nprobe)
    kw = dict(policy=policy, bits=bits, probes=g["probes"][ROWS])
    if policy == "adaptive":
        kw["model"] = mid_full["model"]
    ref = oracle.search(idx, Qs, w.k, w.nprobe, **kw)
    sub = {key: g[key][ROWS] for key in ("ids", "dist", "qdist", "probes")}
    if policy == "fp32":
        compare_fp32(sub, ref, idx, Qs)
    else:
        assert np.array_equal(g["bits"][ROWS], ref["bits"])
        compare_integer(sub, ref)
