"""GPU serving loop (amp_server_*): continuously batched single-query
requests return exactly what a search of that query alone returns (and the
oracle's result for it), admission rejects beyond the request pool, cancel
and callbacks behave as declared, statistics count what happened."""
import threading
import time

import numpy as np
import pytest

import oracle
import paper_2606_07156_amd as amp
from amp_data import build_index
from amp_data.synth import WORKLOADS, make_base, make_queries
from _parity import compare_integer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    w = WORKLOADS["tiny"]
    base = make_base(w)
    idx = build_index(base, w.nlist, w.M, iters=10, seed=w.seed)
    h = amp.amp_index_from_arrays(idx)
    amp.amp_index_to_device(h, 0)
    return dict(idx=idx, h=h, Q=make_queries(w, 160))


def _bufs(n, kmax):
    return (np.full((n, kmax), -7, np.int64), np.full((n, kmax), np.nan, np.float32),
            np.full((n, kmax), -7, np.int64))


def test_mixed_requests_equal_single_query_searches_and_the_oracle(ctx):
    Q = ctx["Q"]
    r = np.random.default_rng(1)
    ks = r.choice([1, 5, 10, 50], size=len(Q)).astype(np.int32)
    nps = r.integers(1, 17, size=len(Q)).astype(np.int32)
    srv = amp.amp_server_create(ctx["h"], max_batch=32, max_pending=256, max_k=50, max_nprobe=16, policy="fixed",
                                bits=8)
    ids, dist, qd = _bufs(len(Q), 50)
    done = []
    for i in range(len(Q)):
        amp.amp_server_submit(srv, Q[i], ks[i], nps[i], ids[i], dist[i], qd[i], done=done.append)
    amp.amp_server_flush(srv)
    assert done == [amp.AMP_OK] * len(Q)
    st = amp.amp_server_stats(srv)
    assert st["completed"] == len(Q) and st["rejected"] == 0 and st["failed"] == 0
    assert st["batches"] >= len(Q) // 32 and st["p50_ms"] > 0 and st["p99_ms"] >= st["p50_ms"]
    for i in range(0, len(Q), 7):
        one = amp.amp_search(ctx["h"], Q[i:i + 1], int(ks[i]), int(nps[i]), policy="fixed", bits=8)
        k = ks[i]
        assert np.array_equal(ids[i, :k], one["ids"][0]) and np.array_equal(qd[i, :k], one["qdist"][0])
        assert np.array_equal(dist[i, :k].view(np.uint32), one["dist"][0].view(np.uint32))
        assert (ids[i, k:] == -7).all()  # beyond k: untouched
    g = amp.amp_search(ctx["h"], Q, ks, nps, policy="fixed", bits=8, want_probes=True)
    ref = oracle.search(ctx["idx"], Q, ks, nps, probes=g["probes"], policy="fixed", bits=8)
    got = dict(ids=np.full_like(ref["ids"], -1), qdist=np.full_like(ref["qdist"], np.iinfo(np.int64).max),
               dist=np.full_like(ref["dist"], np.inf))
    for i in range(len(Q)):
        got["ids"][i, :ks[i]], got["qdist"][i, :ks[i]], got["dist"][i, :ks[i]] = ids[i, :ks[i]], qd[i, :ks[i]], dist[i, :ks[i]]
    compare_integer(got, ref)
    srv.close()


def test_per_request_policies_are_batched_apart(ctx):
    Q = ctx["Q"][:40]
    srv = amp.amp_server_create(ctx["h"], max_batch=16, max_k=10, max_nprobe=8, policy="fixed", bits=16)
    p4 = amp.make_policy("fixed", 4)
    ids, dist, qd = _bufs(len(Q), 10)
    for i in range(len(Q)):
        amp.amp_server_submit(srv, Q[i], 10, 8, ids[i], dist[i], qd[i], policy=p4 if i % 3 == 0 else None)
    amp.amp_server_flush(srv)
    a16 = amp.amp_search(ctx["h"], Q, 10, 8, policy="fixed", bits=16)
    a4 = amp.amp_search(ctx["h"], Q, 10, 8, policy="fixed", bits=4)
    for i in range(len(Q)):
        want = a4 if i % 3 == 0 else a16
        assert np.array_equal(ids[i], want["ids"][i]) and np.array_equal(qd[i], want["qdist"][i])
    srv.close()


def test_admission_rejects_beyond_the_request_pool_and_cancel(ctx):
    Q = ctx["Q"]
    # a one-second batch window holds the first requests in the pool
    srv = amp.amp_server_create(ctx["h"], max_batch=64, max_pending=4, max_k=10, max_nprobe=8,
                                batch_window_us=1_000_000, policy="fixed", bits=12)
    ids, dist, qd = _bufs(6, 10)
    seen = {}
    t = [amp.amp_server_submit(srv, Q[i], 10, 8, ids[i], dist[i], qd[i],
                               done=lambda st, i=i: seen.__setitem__(i, st)) for i in range(4)]
    with pytest.raises(amp.AmpError) as e:
        amp.amp_server_submit(srv, Q[4], 10, 8, ids[4], dist[4], qd[4])
    assert e.value.status == amp.AMP_EBUSY
    amp.amp_server_cancel(srv, t[1])
    assert seen.get(1) == amp.AMP_ECANCELED  # queued: cancelled at once
    with pytest.raises(amp.AmpError) as e:
        amp.amp_server_cancel(srv, t[1])
    assert e.value.status == amp.AMP_EINVAL
    # the cancelled request's slot is free again
    amp.amp_server_submit(srv, Q[5], 10, 8, ids[5], dist[5], qd[5])
    amp.amp_server_flush(srv)
    assert seen == {0: 0, 1: amp.AMP_ECANCELED, 2: 0, 3: 0}
    assert (ids[1] == -7).all() and (ids[4] == -7).all()
    ref = amp.amp_search(ctx["h"], Q[:6], 10, 8, policy="fixed", bits=12)
    for i in (0, 2, 3, 5):
        assert np.array_equal(ids[i], ref["ids"][i]) and np.array_equal(qd[i], ref["qdist"][i])
    st = amp.amp_server_stats(srv, reset=True)
    assert (st["submitted"], st["rejected"], st["completed"], st["cancelled"]) == (6, 1, 4, 1)
    assert st["batches"] == 1 and st["mean_batch"] == 4  # the window gathered them into one launch
    st = amp.amp_server_stats(srv)
    assert st["submitted"] == 0 and st["completed"] == 0 and st["p99_ms"] == 0
    srv.close()


def test_invalid_requests_queue_nothing(ctx):
    srv = amp.amp_server_create(ctx["h"], max_batch=8, max_k=10, max_nprobe=8)
    ids, dist, qd = _bufs(1, 20)
    for kw, frag in [(dict(k=11, nprobe=2), "k = 11"), (dict(k=3, nprobe=9), "nprobe = 9"),
                     (dict(k=3, nprobe=2, policy=amp.make_policy("adaptive")), "predictor")]:
        with pytest.raises(amp.AmpError) as e:
            amp.amp_server_submit(srv, ctx["Q"][0], out_ids=ids[0], out_dist=dist[0], **kw)
        assert e.value.status == amp.AMP_EINVAL and frag in str(e.value)
    assert amp.amp_server_stats(srv)["submitted"] == 0
    srv.close()


def test_concurrent_submitters_and_destroy_drains(ctx):
    Q = ctx["Q"]
    srv = amp.amp_server_create(ctx["h"], max_batch=24, max_pending=256, max_k=10, max_nprobe=8, policy="fixed",
                                bits=16)
    ids, dist, qd = _bufs(len(Q), 10)
    count = []

    def feed(lo, hi):
        for i in range(lo, hi):
            amp.amp_server_submit(srv, Q[i], 10, 8, ids[i], dist[i], qd[i], done=count.append,
                                  arrival_ns=time.monotonic_ns())

    th = [threading.Thread(target=feed, args=(j * 40, (j + 1) * 40)) for j in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    srv.close()  # drains every admitted request before it returns
    assert len(count) == len(Q) and set(count) == {amp.AMP_OK}
    ref = amp.amp_search(ctx["h"], Q, 10, 8, policy="fixed", bits=16)
    assert np.array_equal(ids, ref["ids"]) and np.array_equal(qd, ref["qdist"])


def test_bf16_server_equals_fp32_search_of_the_widened_queries(ctx):
    from _parity import bf16_bits, bf16_widen
    Qb = bf16_bits(ctx["Q"][:50])
    srv = amp.amp_server_create(ctx["h"], max_batch=16, max_k=10, max_nprobe=8, q_dtype="bf16",
                                policy="fixed", bits=8)
    ids, dist, qd = _bufs(len(Qb), 10)
    for i in range(len(Qb)):
        amp.amp_server_submit(srv, Qb[i], 10, 8, ids[i], dist[i], qd[i])
    amp.amp_server_flush(srv)
    ref = amp.amp_search(ctx["h"], bf16_widen(Qb), 10, 8, policy="fixed", bits=8)
    assert np.array_equal(ids, ref["ids"]) and np.array_equal(qd, ref["qdist"])
    srv.close()


def test_a_batch_whose_search_overflows_fails_with_the_device_status(ctx, monkeypatch):
    # a 64-entry candidate buffer and no re-runs: a 4-bit batch overflows on
    # the device; its requests complete with AMP_EOVERFLOW (not with wrong ids)
    monkeypatch.setenv("AMP_CAPQ", "64")
    monkeypatch.setenv("AMP_RERUNS", "0")
    Q = ctx["Q"][:24]
    srv = amp.amp_server_create(ctx["h"], max_batch=32, max_k=10, max_nprobe=8, policy="fixed", bits=4,
                                batch_window_us=20000)
    ids, dist, qd = _bufs(len(Q), 10)
    done = []
    for i in range(len(Q)):
        amp.amp_server_submit(srv, Q[i], 10, 8, ids[i], dist[i], qd[i], done=done.append)
    amp.amp_server_flush(srv)
    assert amp.AMP_EOVERFLOW in done and set(done) <= {amp.AMP_OK, amp.AMP_EOVERFLOW}
    st = amp.amp_server_stats(srv)
    assert st["failed"] == done.count(amp.AMP_EOVERFLOW)
    srv.close()


@pytest.fixture(scope="module")
def wide():
    # the serving shape (d 768 unit vectors, inner product, PQ96) with 512
    # lists, so that nprobe reaches 256; a predictor spread over the widths
    import dataclasses
    from test_gpu_parity import _spread_model
    w = dataclasses.replace(WORKLOADS["serving"], n=40_000, nq=48, nlist=512, nprobe=256)
    base = make_base(w)
    idx = build_index(base, w.nlist, w.M, iters=8, seed=w.seed, grid_kind=w.grid_kind, metric=w.metric)
    h = amp.amp_index_from_arrays(idx)
    amp.amp_index_to_device(h, 0)
    c = dict(idx=idx, h=h, Q=make_queries(w, 48))
    m = _spread_model(c, 64, seed=5)
    amp.amp_index_set_predictor(h, m)
    c["model"] = m
    return c


def test_adaptive_inner_product_mix_equals_each_request_alone(wide):
    """ADAPTIVE under inner product with k in {10, 50, 100} and nprobe in
    {16, 64, 256}: every request's result in the continuously batched mix
    (two batches in flight on their own streams) equals the search of that
    query alone, and the oracle's for it."""
    Q = wide["Q"]
    r = np.random.default_rng(8)
    ks = r.choice([10, 50, 100], size=len(Q)).astype(np.int32)
    nps = r.choice([16, 64, 256], size=len(Q)).astype(np.int32)
    srv = amp.amp_server_create(wide["h"], max_batch=8, max_pending=64, max_k=100, max_nprobe=256,
                                policy="adaptive")
    ids, dist, qd = _bufs(len(Q), 100)
    done = []
    for i in range(len(Q)):
        amp.amp_server_submit(srv, Q[i], ks[i], nps[i], ids[i], dist[i], qd[i], done=done.append)
    amp.amp_server_flush(srv)
    assert done == [amp.AMP_OK] * len(Q)
    assert amp.amp_server_stats(srv)["batches"] >= len(Q) // 8
    for i in range(len(Q)):
        one = amp.amp_search(wide["h"], Q[i:i + 1], int(ks[i]), int(nps[i]), policy="adaptive", want_probes=True)
        k = ks[i]
        assert np.array_equal(ids[i, :k], one["ids"][0]), i
        assert np.array_equal(qd[i, :k], one["qdist"][0]), i
        assert np.array_equal(dist[i, :k].view(np.uint32), one["dist"][0].view(np.uint32)), i
        if i % 6 == 0:
            ref = oracle.search(wide["idx"], Q[i:i + 1], int(k), int(nps[i]), probes=one["probes"],
                                policy="adaptive", model=wide["model"])
            compare_integer(one, ref)
    srv.close()
