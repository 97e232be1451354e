"""GPU index builder (amp_index_build, Sec. 2.1): the arrays it returns are
checked against what the construction defines, recomputed in FP64 from the
base vectors: every vector in its nearest list, every code the nearest
codeword of its residual (FP32 near-ties certified), lists partitioning the
ids in increasing order, radius and grid step by their definitions, one
Lloyd step exactly the mean of its clusters, and searches on the built index
bit-exact against the oracle."""
import numpy as np
import pytest

import oracle
import paper_2606_07156_amd as amp
from amp_data import build_index
from amp_data.synth import WORKLOADS, make_base, make_queries
from _parity import certify_probes, compare_integer

pytestmark = pytest.mark.gpu

F64 = np.float64


def _build(base, nlist, M, **kw):
    h = amp.amp_index_build(base, nlist, M, **kw)
    return h, amp.amp_index_get_arrays(h)


@pytest.fixture(scope="module")
def tinyb():
    w = WORKLOADS["tiny"]
    base = make_base(w)
    h, idx = _build(base, w.nlist, w.M, iters=10, seed=7)
    return dict(w=w, base=base, h=h, idx=idx)


def _rows_by_list(idx):
    """base row of every position (the default ids are row numbers)"""
    return np.asarray(idx["ids"])


def _nearest_ok(X, C, chosen):
    """chosen[i] is a nearest row of C to X[i] up to the FP32 expansion
    error |x|^2 + |c|^2 - 2 x.c; returns the number of certified near-ties"""
    X64, C64 = X.astype(F64), C.astype(F64)
    xn = (X64 * X64).sum(1)
    cn = (C64 * C64).sum(1)
    ties = 0
    for s in range(0, len(X), 4096):
        G = X64[s:s + 4096] @ C64.T
        D = xn[s:s + 4096, None] + cn[None, :] - 2 * G
        tol = (X.shape[1] + 4) * 2.0 ** -23 * (xn[s:s + 4096, None] + cn[None, :] + 2 * np.abs(G))
        ch = chosen[s:s + 4096]
        dmin = D.min(1)
        dch = D[np.arange(len(ch)), ch]
        bad = dch > dmin
        if bad.any():
            am = D.argmin(1)
            lim = tol[np.arange(len(ch)), ch] + tol[np.arange(len(ch)), am]
            assert np.all(dch[bad] - dmin[bad] <= lim[bad]), "assignment is not the nearest"
            ties += int(bad.sum())
    return ties


def test_lists_partition_the_ids_in_increasing_order(tinyb):
    idx, n = tinyb["idx"], len(tinyb["base"])
    off = idx["list_offsets"]
    assert off[0] == 0 and off[-1] == n and np.all(np.diff(off) >= 0)
    assert np.array_equal(np.sort(idx["ids"]), np.arange(n))
    for p in range(idx["nlist"]):
        assert np.all(np.diff(idx["ids"][off[p]:off[p + 1]]) > 0)
    assert idx["codes"].shape == (n, idx["M"]) and idx["codebook"].shape == (idx["M"], 256, idx["dsub"])


def test_every_vector_is_in_its_nearest_list(tinyb):
    idx, base = tinyb["idx"], tinyb["base"]
    rows = _rows_by_list(idx)
    lst = np.repeat(np.arange(idx["nlist"]), np.diff(idx["list_offsets"]))
    ties = _nearest_ok(base[rows], idx["centroids"], lst)
    assert ties <= len(base) // 1000


def test_every_code_is_the_nearest_codeword(tinyb):
    idx, base = tinyb["idx"], tinyb["base"]
    rows = _rows_by_list(idx)
    lst = np.repeat(np.arange(idx["nlist"]), np.diff(idx["list_offsets"]))
    R = base[rows] - idx["centroids"][lst]  # FP32 residual, as stored vectors see it
    ds = idx["dsub"]
    ties = 0
    for m in range(idx["M"]):
        ties += _nearest_ok(np.ascontiguousarray(R[:, m * ds:(m + 1) * ds]), idx["codebook"][m],
                            idx["codes"][:, m].astype(np.int64))
    assert ties <= len(base) * idx["M"] // 1000


def test_radius_and_grid_step_follow_their_definitions(tinyb):
    idx, base = tinyb["idx"], tinyb["base"]
    rows = _rows_by_list(idx)
    off = idx["list_offsets"]
    lst = np.repeat(np.arange(idx["nlist"]), np.diff(off))
    R = (base[rows] - idx["centroids"][lst]).astype(F64)
    A = max(np.abs(R).max(), np.abs(idx["codebook"]).max())
    e = idx["grid_e"]
    assert A / 2.0 ** e <= 255 < A / 2.0 ** (e - 1)
    rn = np.sqrt((R * R).sum(1))
    rad = np.zeros(idx["nlist"])
    np.maximum.at(rad, lst, rn)
    assert np.all(np.abs(idx["radq"] - rad / 2.0 ** e) <= 0.5 + 1e-9)


def test_one_lloyd_step_is_the_mean_of_its_clusters():
    # n <= 256 * nlist: k-means trains on every vector; zero iterations leave
    # the seeded distinct initial points, one iteration replaces each by the
    # mean of the vectors nearest to it
    w = WORKLOADS["tiny"]
    base = make_base(w)[:12_000]
    _, i0 = _build(base, 64, 8, iters=0, seed=3)
    _, i1 = _build(base, 64, 8, iters=1, seed=3)
    C0, C1 = i0["centroids"], i1["centroids"]
    assert len(np.unique(C0, axis=0)) == 64
    for c in C0:  # initial centroids are base rows
        assert (np.abs(base - c).max(1) == 0).any()
    X64, C064 = base.astype(F64), C0.astype(F64)
    xn, cn = (X64 * X64).sum(1), (C064 * C064).sum(1)
    G = X64 @ C064.T
    D = xn[:, None] + cn[None, :] - 2 * G
    a = D.argmin(1)
    # rows whose nearest centroid an FP32 evaluation may pick differently
    tol = 2 * (base.shape[1] + 4) * 2.0 ** -23 * (xn[:, None] + cn[None, :] + 2 * np.abs(G))
    amb = (D - D.min(1, keepdims=True)) <= tol
    ambiguous = amb.sum(1) > 1
    touched = set(np.flatnonzero(amb[ambiguous].any(0)).tolist())
    checked = 0
    for c in range(64):
        mem = a == c
        if not mem.any() or c in touched:
            continue
        mean = X64[mem].mean(0)
        assert np.allclose(C1[c], mean, rtol=1e-6, atol=1e-6 * np.abs(base).max()), c
        checked += 1
    assert checked >= 48


def test_build_is_deterministic_and_keeps_caller_ids(tinyb):
    base, w = tinyb["base"], tinyb["w"]
    _, again = _build(base, w.nlist, w.M, iters=10, seed=7)
    for key in ("centroids", "codebook", "list_offsets", "ids", "codes", "radq"):
        assert np.array_equal(again[key], tinyb["idx"][key]), key
    assert again["grid_e"] == tinyb["idx"]["grid_e"]
    r = np.random.default_rng(5)
    cid = (10 ** 12 + r.permutation(len(base))).astype(np.int64)
    _, ci = _build(base, w.nlist, w.M, iters=10, seed=7, ids=cid)
    off = ci["list_offsets"]
    assert np.array_equal(off, tinyb["idx"]["list_offsets"])
    rows = _rows_by_list(tinyb["idx"])
    for p in range(w.nlist):
        got = ci["ids"][off[p]:off[p + 1]]
        assert np.all(np.diff(got) > 0)
        assert np.array_equal(got, np.sort(cid[rows[off[p]:off[p + 1]]]))


def test_quality_matches_the_reference_builder(tinyb):
    # same construction with other seeded samples: the coarse and PQ
    # quantisation errors agree within a few percent
    w, base = tinyb["w"], tinyb["base"]
    ref = build_index(base, w.nlist, w.M, iters=10, seed=7)

    def errors(idx):
        rows = _rows_by_list(idx)
        lst = np.repeat(np.arange(idx["nlist"]), np.diff(idx["list_offsets"]))
        R = base[rows].astype(F64) - idx["centroids"][lst]
        rec = np.concatenate([idx["codebook"][m][idx["codes"][:, m]] for m in range(idx["M"])], 1)
        return (R * R).sum(1).mean(), ((R - rec) ** 2).sum(1).mean()

    ec, ep = errors(tinyb["idx"])
    rc, rp = errors(ref)
    assert ec <= 1.08 * rc and ep <= 1.08 * rp, (ec, rc, ep, rp)


@pytest.mark.parametrize("bits", [8, 16])
def test_search_on_the_built_index_matches_the_oracle(tinyb, bits):
    Q = make_queries(tinyb["w"], 64)
    g = amp.amp_search(tinyb["h"], Q, 10, 8, policy="fixed", bits=bits, want_probes=True)
    certify_probes(g["probes"], tinyb["idx"], Q, 8)
    ref = oracle.search(tinyb["idx"], Q, 10, 8, probes=g["probes"], policy="fixed", bits=bits)
    compare_integer(g, ref)


def test_integer_data_build_is_on_the_unit_grid():
    w = WORKLOADS["mid"].scaled(n=30_000, nq=32, nlist=64)
    base = make_base(w)
    h, idx = _build(base, 64, w.M, iters=6, seed=2, integer_data=True)
    assert idx["grid_e"] == 0
    assert np.array_equal(idx["centroids"], np.rint(idx["centroids"]))
    assert np.array_equal(idx["codebook"], np.rint(idx["codebook"]))
    lst = np.repeat(np.arange(64), np.diff(idx["list_offsets"]))
    _nearest_ok(base[idx["ids"]], idx["centroids"], lst)
    Q = make_queries(w, 32)
    g = amp.amp_search(h, Q, 10, 8, policy="fixed", bits=12, want_probes=True)
    ref = oracle.search(idx, Q, 10, 8, probes=g["probes"], policy="fixed", bits=12)
    compare_integer(g, ref)


def test_inner_product_e4m3_build_grid_covers_vectors_and_centroids():
    w = WORKLOADS["serving"].scaled(n=20_000, nq=32, nlist=64)
    base = make_base(w)
    h, idx = _build(base, 64, 96, iters=6, seed=4, metric="ip", grid_kind="e4m3")
    lst = np.repeat(np.arange(64), np.diff(idx["list_offsets"]))
    R = base[idx["ids"]].astype(F64) - idx["centroids"][lst]
    A = max(np.abs(R).max(), np.abs(idx["codebook"]).max(), np.abs(idx["centroids"]).max(), np.abs(base).max())
    e = idx["grid_e"]
    assert A / 2.0 ** e <= 448 < A / 2.0 ** (e - 1)
    Q = make_queries(w, 32)
    g = amp.amp_search(h, Q, 20, 8, policy="fixed", bits=8, want_probes=True)
    ref = oracle.search(idx, Q, 20, 8, probes=g["probes"], policy="fixed", bits=8)
    compare_integer(g, ref)


def test_few_distinct_vectors_leave_empty_lists():
    r = np.random.default_rng(9)
    distinct = r.integers(-20, 20, size=(10, 16)).astype(np.float32)
    base = distinct[r.integers(0, 10, size=300)]
    h, idx = _build(base, 16, 4, iters=4, seed=1, integer_data=True)
    sizes = np.diff(idx["list_offsets"])
    assert sizes.sum() == 300 and (sizes > 0).sum() <= 10
    lst = np.repeat(np.arange(16), sizes)
    _nearest_ok(base[idx["ids"]], idx["centroids"], lst)
    Q = distinct[:4] + 0.0
    g = amp.amp_search(h, Q, 5, 4, policy="fixed", bits=16, want_probes=True)
    ref = oracle.search(idx, Q, 5, 4, probes=g["probes"], policy="fixed", bits=16)
    compare_integer(g, ref)


def test_bf16_base_builds_the_index_of_its_fp32_values():
    from _parity import bf16_bits, bf16_widen
    w = WORKLOADS["tiny"]
    b16 = bf16_bits(make_base(w)[:8000])
    _, a = _build(b16, 32, 8, iters=4, seed=11)
    _, b = _build(bf16_widen(b16), 32, 8, iters=4, seed=11)
    for key in ("centroids", "codebook", "list_offsets", "ids", "codes", "radq"):
        assert np.array_equal(a[key], b[key]), key
    assert a["grid_e"] == b["grid_e"]
