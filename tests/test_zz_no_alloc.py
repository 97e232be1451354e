"""The allocation-free entry point amp_search_noalloc through the C ABI: its
results equal amp_search's (bit for bit: the same kernels on the same
inputs, only the scratch and the list chunking differ) on two calls in a
row, the second with a smaller batch, under integer and full-precision
policies, with constant and device-resident per-query sizes."""
import numpy as np
import pytest

import paper_2606_07156_amd as amp
from amp_data import build_index
from amp_data.synth import WORKLOADS, make_base, make_queries

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from test_gpu_parity import _spread_model
    w = WORKLOADS["tiny"]
    base = make_base(w)
    idx = build_index(base, w.nlist, w.M, iters=10, seed=w.seed)
    h = amp.amp_index_from_arrays(idx)
    c = dict(idx=idx, h=h, Q=make_queries(w, 100))
    amp.amp_index_set_predictor(h, _spread_model(c, 8))
    amp.amp_index_to_device(h, 0)  # resident with its predictor: nothing left to allocate
    return c


def _outs(torch, nq, kmax):
    return dict(ids=torch.full((nq, kmax), -7, dtype=torch.int64, device="cuda"),
                dist=torch.full((nq, kmax), -7.0, dtype=torch.float32, device="cuda"),
                qdist=torch.full((nq, kmax), -7, dtype=torch.int64, device="cuda"),
                status=torch.full((1,), 12345, dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("policy,bits", [("fixed", 8), ("fixed", 16), ("adaptive", 0), ("fp32", 0)])
def test_noalloc_equals_amp_search_on_two_calls(ctx, policy, bits):
    torch = pytest.importorskip("torch")
    s = torch.cuda.Stream()
    Q = ctx["Q"]
    for nq in (100, 37):  # the second call smaller than the first
        qd = torch.from_numpy(np.ascontiguousarray(Q[:nq])).cuda()
        a = _outs(torch, nq, 10)
        b = _outs(torch, nq, 10)
        amp.amp_search(ctx["h"], qd, 10, 8, policy=policy, bits=bits, out=a, stream=s)
        amp.amp_search_noalloc(ctx["h"], qd, 10, 8, policy=policy, bits=bits, out=b, stream=s)
        s.synchronize()
        assert int(b["status"].item()) == amp.AMP_OK
        for key in ("ids", "qdist"):
            assert np.array_equal(a[key].cpu().numpy(), b[key].cpu().numpy()), (nq, key)
        assert np.array_equal(a["dist"].cpu().numpy().view(np.uint32), b["dist"].cpu().numpy().view(np.uint32))


def test_noalloc_with_device_sizes_on_two_calls(ctx):
    torch = pytest.importorskip("torch")
    s = torch.cuda.Stream()
    Q = ctx["Q"]
    r = np.random.default_rng(3)
    for nq in (64, 20):
        ks = r.integers(1, 21, size=nq).astype(np.int32)
        nps = r.integers(1, 13, size=nq).astype(np.int32)
        qd = torch.from_numpy(np.ascontiguousarray(Q[:nq])).cuda()
        kd, npd = torch.from_numpy(ks).cuda(), torch.from_numpy(nps).cuda()
        b = _outs(torch, nq, 20)
        amp.amp_search_noalloc(ctx["h"], qd, kd, npd, kmax=20, npmax=12, policy="fixed", bits=4, out=b, stream=s)
        s.synchronize()
        assert int(b["status"].item()) == amp.AMP_OK
        want = amp.amp_search(ctx["h"], Q[:nq], ks, nps, policy="fixed", bits=4)
        got = b["ids"].cpu().numpy()
        gq = b["qdist"].cpu().numpy()
        for i in range(nq):
            assert np.array_equal(got[i, :ks[i]], want["ids"][i, :ks[i]]), (nq, i)
            assert np.array_equal(gq[i, :ks[i]], want["qdist"][i, :ks[i]]), (nq, i)


def test_noalloc_rejections(ctx):
    torch = pytest.importorskip("torch")
    qd = torch.from_numpy(ctx["Q"][:4]).cuda()
    o = _outs(torch, 4, 10)
    s = torch.cuda.Stream()
    with pytest.raises(amp.AmpError):  # per-query host arrays
        amp.amp_search_noalloc(ctx["h"], qd, [10, 5, 10, 5], 8, out=o, stream=s)
    with pytest.raises(amp.AmpError):  # host memory
        amp.amp_search_noalloc(ctx["h"], ctx["Q"][:4], 10, 8)
    with pytest.raises(amp.AmpError) as e:  # does not fit the fixed scratch
        big = torch.zeros((1 << 16, ctx["Q"].shape[1]), dtype=torch.float32, device="cuda")
        amp.amp_search_noalloc(ctx["h"], big, 1024, 64, out=_outs(torch, 1 << 16, 1024), stream=s)
    assert e.value.status == amp.AMP_EINVAL
