"""Host side of reduced-precision cluster locating: the sub-space map the
library builds (codes, slices, nearest-centre partition, radius, count)
checked against its definition by brute force, and the CL predictor's
trainer end to end.  CPU only."""
import numpy as np
import pytest

import oracle
import paper_2606_07156_amd as amp
from amp_data import build_index
from amp_data.synth import WORKLOADS, make_base, make_queries
from oracle import cl as ocl


@pytest.fixture(scope="module")
def small():
    w = WORKLOADS["mid"].scaled(n=40_000, nlist=96)
    base = make_base(w)
    idx = build_index(base, w.nlist, w.M, iters=6, seed=w.seed, integer_data=True)
    h = amp.amp_index_from_arrays(idx)
    return dict(w=w, idx=idx, h=h)


def _check_map(idx, m, S, P):
    C = np.asarray(idx["centroids"], np.float32)
    d = C.shape[1]
    o, ec = ocl.cl_params(C, idx["metric"])
    assert m["S"] == S and m["P"] == P and m["w"] == d // S
    assert m["o"] == o and m["ec"] == ec
    V = ocl.cl_codes(C, o, ec)
    assert V.min() >= -128 and V.max() <= 127
    for s, (a, b) in enumerate(ocl.slices(d, S)):
        Z = m["centre"][s]
        d2 = ((V[:, None, a:b] - Z[None, :, :]) ** 2).sum(-1)  # [nlist, P]
        # nearest rounded centre, ties to the lower index (first minimum)
        assert np.array_equal(m["assign"][:, s], d2.argmin(1)), s
        assert np.array_equal(m["count"][s], np.bincount(m["assign"][:, s], minlength=P)), s
        for u in range(P):
            mem = d2[m["assign"][:, s] == u, u]
            r2 = int(mem.max()) if len(mem) else 0
            r = int(m["radius"][s, u])
            assert r * r >= r2 and (r == 0 or (r - 1) * (r - 1) < r2), (s, u)


@pytest.mark.parametrize("S,P", [(16, 32), (8, 96), (4, 7)])
def test_map_is_the_nearest_centre_partition(small, S, P):
    amp.amp_index_build_cl_map(small["h"], S, P, iters=10, seed=3)
    m = amp.amp_index_get_cl_map(small["h"])
    _check_map(small["idx"], m, S, P)
    assert np.array_equal(m["count"].sum(1), np.full(S, small["idx"]["nlist"]))


def test_map_inner_product_offset_zero():
    from amp_data.synth import Workload
    w = Workload("t", 8000, 96, 48, 16, 40, 12, 8, 10, "vmf", 5, metric="ip")
    base = make_base(w)
    idx = build_index(base, 40, 12, iters=5, seed=5, metric="ip")
    h = amp.amp_index_from_arrays(idx)
    amp.amp_index_build_cl_map(h, 12, 10, iters=8, seed=1)
    m = amp.amp_index_get_cl_map(h)
    assert m["o"] == 0
    _check_map(idx, m, 12, 10)


def test_map_arguments_are_checked(small):
    h = small["h"]
    for S, P in ((3, 8), (0, 8), (16, 0), (16, 97), (1, 8)):  # d % S, S 0, P 0, P > nlist, d / S > 64
        with pytest.raises(amp.AmpError):
            amp.amp_index_build_cl_map(h, S, P)
    # a CL predictor needs a map
    model = dict(n_sv=0, sv=np.zeros((0, 5)), beta=np.zeros(0), table=np.zeros(1024), beta0=0,
                 feat_lo=[0] * 5, feat_mul=[0] * 5, g_mul=0, theta=[0, 0, 0])
    with pytest.raises(amp.AmpError):
        amp.amp_index_set_cl_predictor(amp.amp_index_from_arrays(small["idx"]), model)


def test_cl_trainer_end_to_end(small):
    h, w, idx = small["h"], small["w"], small["idx"]
    amp.amp_index_build_cl_map(h, 16, 24, iters=10, seed=0)
    TQ = make_queries(w, 48, train=True)
    rep = amp.amp_index_train_cl_predictor(h, TQ, 8, low=4, n_samples=600)
    m = amp.amp_index_get_cl_map(h)
    nonempty = int((m["count"] > 0).sum())
    assert rep["n_pairs"] == 48 * nonempty and sum(rep["label_hist"]) == rep["n_pairs"]
    assert 0 < rep["n_sv"] <= rep["n_samples"] <= 600
    model = amp.amp_index_get_cl_predictor(h)
    assert model["n_sv"] == rep["n_sv"] and model["theta"][0] == 1 << 39
    # the oracle evaluates the trained model on fresh queries: widths are 4 or
    # 8, both occur
    Q = make_queries(w, 6)
    share = []
    for q in Q:
        vq = ocl.cl_codes(q, m["o"], m["ec"])
        bits, _ = ocl.predict_cl_bits(vq, m, model, 4)
        assert set(np.unique(bits)) <= {4, 8}
        share.append(ocl.low_share(bits, m, 4))
    assert 0 < np.mean(share) < 1
    # rebuilding the map drops the CL predictor
    amp.amp_index_build_cl_map(h, 16, 24, iters=10, seed=0)
    with pytest.raises(amp.AmpError):
        amp.amp_index_get_cl_predictor(h)


def test_map_and_cl_predictor_survive_save_and_load(small, tmp_path):
    h = small["h"]
    amp.amp_index_build_cl_map(h, 8, 20, iters=5, seed=4)
    amp.amp_index_train_cl_predictor(h, make_queries(small["w"], 24, train=True), 8, low=3, n_samples=200)
    path = str(tmp_path / "cl.ampidx")
    amp.amp_index_save(h, path)
    h2 = amp.amp_index_load(path)
    m1, m2 = amp.amp_index_get_cl_map(h), amp.amp_index_get_cl_map(h2)
    for key in ("S", "P", "w", "o", "ec"):
        assert m1[key] == m2[key], key
    for key in ("assign", "centre", "radius", "count"):
        assert np.array_equal(m1[key], m2[key]), key
    p1, p2 = amp.amp_index_get_cl_predictor(h), amp.amp_index_get_cl_predictor(h2)
    for key in ("sv", "beta", "table", "feat_lo", "feat_mul", "theta"):
        assert np.array_equal(p1[key], p2[key]), key
    assert p1["beta0"] == p2["beta0"] and p1["g_mul"] == p2["g_mul"]
