"""Predictor training (host): the SVR solver against scikit-learn's SVR on the
same precomputed kernel, and the trainer end to end on a small index."""
import numpy as np
import pytest

import oracle
import paper_2606_07156_amd as amp
from amp_data import build_index
from amp_data.synth import WORKLOADS, make_base, make_queries


def _rbf(X, gamma):
    d2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    return np.exp(-gamma * d2)


@pytest.mark.parametrize("C,eps", [(1.0, 0.05), (10.0, 0.1), (0.5, 0.01)])
def test_svr_solver_matches_sklearn(C, eps):
    """Same dual optimum as libsvm's epsilon-SVR (scikit-learn, an independent
    implementation) within the solvers' tolerances."""
    svm = pytest.importorskip("sklearn.svm")
    r = np.random.default_rng(3)
    X = r.uniform(0, 1, size=(150, 5))
    y = (np.sin(4 * X[:, 0]) + X[:, 1] ** 2 > 0.8).astype(float) + 0.05 * r.normal(size=150)
    K = _rbf(X, 2.0)
    coef, b, it = amp.amp_svr_fit(K, y, C_=C, epsilon=eps, tol=1e-6, max_iter=2_000_000)
    ref = svm.SVR(kernel="precomputed", C=C, epsilon=eps, tol=1e-6).fit(K, y)
    ref_coef = np.zeros(len(y))
    ref_coef[ref.support_] = ref.dual_coef_[0]
    assert np.abs(coef).max() <= C + 1e-9
    assert abs(coef.sum()) < 1e-8
    f = K @ coef + b
    f_ref = ref.predict(K)
    assert np.abs(f - f_ref).max() < 2e-3
    assert np.abs(coef - ref_coef).max() < 5e-2 * C


def test_trainer_end_to_end_on_a_small_index():
    w = WORKLOADS["mid"].scaled(n=60_000, nlist=64)
    base = make_base(w)
    idx = build_index(base, w.nlist, w.M, iters=6, seed=w.seed, integer_data=True)
    h = amp.amp_index_from_arrays(idx)
    TQ = make_queries(w, 64, train=True)
    rep = amp.amp_index_train_predictor(h, TQ, 10, 8, n_samples=400, gamma=10.0, epsilon=0.1)
    assert rep["n_pairs"] == 64 * 8 and sum(rep["label_hist"]) == rep["n_pairs"]
    assert 0 < rep["n_sv"] <= rep["n_samples"] <= 400
    m = amp.amp_index_get_predictor(h)
    assert m["n_sv"] == rep["n_sv"] and m["sv"].min() >= 0 and m["sv"].max() <= 1023
    # the oracle evaluates the trained model: widths are allowed ones, and the
    # nearest probed list tends to get more bits than the farthest
    Q = make_queries(w, 24)
    res = oracle.search(idx, Q, 10, 8, policy="adaptive", model=m)
    b = res["bits"]
    assert set(np.unique(b)) <= {4, 8, 12, 16}
    assert b[:, 0].mean() >= b[:, -1].mean()
    # restricting the widths keeps the choice inside the allowed set
    rep2 = amp.amp_index_train_predictor(h, TQ, 10, 8, n_samples=200, allowed=(4, 16))
    assert rep2["label_hist"][1] == rep2["label_hist"][2] == 0
    # save / load keeps the model
    import tempfile, os
    with tempfile.TemporaryDirectory() as d:
        amp.amp_index_save(h, os.path.join(d, "x.idx"))
        h2 = amp.amp_index_load(os.path.join(d, "x.idx"))
        m2 = amp.amp_index_get_predictor(h2)
        m1 = amp.amp_index_get_predictor(h)
        for key in ("sv", "beta", "table", "feat_lo", "feat_mul", "theta"):
            assert np.array_equal(m1[key], m2[key])
        assert m1["beta0"] == m2["beta0"] and m1["g_mul"] == m2["g_mul"]


def test_trainer_argument_validation():
    w = WORKLOADS["tiny"].scaled(n=5000)
    idx = build_index(make_base(w), 16, 8, iters=3, seed=1)
    h = amp.amp_index_from_arrays(idx)
    TQ = make_queries(w, 4, train=True)
    with pytest.raises(amp.AmpError):
        amp.amp_index_train_predictor(h, TQ, 10, 0)
    with pytest.raises(amp.AmpError):
        amp.amp_index_train_predictor(h, TQ, 10, 4, n_samples=2)
    with pytest.raises(amp.AmpError):
        amp.amp_index_train_predictor(h, TQ, 10, 4, allowed=(4, 6))
    with pytest.raises(amp.AmpError):
        amp.amp_index_get_predictor(h)


def _labels_by_definition(idx, TQ, k, nprobe, widths=(4, 8, 12, 16)):
    """Label histogram of the training pairs, recomputed from the oracle's
    stage functions: exact integer ADC distances on the operand grid; the
    list's margin between the query's k neighbours (by (distance, id)) and
    the other candidates; the smallest width whose worst-case quantisation
    error M * 2^(s-1) stays below that margin (or that needs no shift)."""
    M, metric, kind = int(idx["M"]), idx["metric"], idx["grid_kind"]
    inv = 2.0 ** (-int(idx["grid_e"]))
    cbi, ci = oracle.index_grid(idx)
    C = np.asarray(idx["centroids"], np.float32)
    offs, ids, codes = idx["list_offsets"], idx["ids"], idx["codes"].astype(np.int64)
    hist = [0, 0, 0, 0]
    for q in TQ:
        P = oracle.select_probes(oracle.coarse_distances(q, C, metric), nprobe)
        dists, Ts = [], []
        if metric == "ip":
            qi = oracle.grid(q.astype(np.float64) * inv, kind)
            Tq = oracle.lut_int(qi, cbi, "ip")
        for p in P:
            if metric in ("l2", "l1"):
                T = oracle.lut_int(oracle.grid(oracle.residual_f32(q, C[p]).astype(np.float64) * inv, kind), cbi,
                                   metric)
                extra = 0
            else:
                T, extra = Tq, -int((qi * ci[p]).sum())
            c = codes[offs[p]:offs[p + 1]]
            dists.append(extra + T[np.arange(M)[None, :], c].sum(1))
            Ts.append(T)
        allv = sorted((int(v), int(i)) for r, p in enumerate(P) for v, i in zip(dists[r], ids[offs[p]:offs[p + 1]]))
        if len(allv) <= k:
            continue
        kth, dk, dk1 = allv[k - 1], allv[k - 1][0], allv[k][0]
        for r, p in enumerate(P):
            delta = min((dk1 - v if (int(v), int(i)) <= kth else v - dk)
                        for v, i in zip(dists[r], ids[offs[p]:offs[p + 1]]))
            b_star = widths[-1]
            for b in widths:
                s = oracle.quantize_lut(Ts[r], b)[1]
                if s == 0 or M * (1 << (s - 1)) < delta:
                    b_star = b
                    break
            hist[b_star // 4 - 1] += 1
    return hist


@pytest.mark.parametrize("metric", ["l2", "ip", "l1"])
def test_trainer_labels_follow_the_margin_definition(metric):
    w = WORKLOADS["tiny"].scaled(n=6000)
    base = make_base(w)
    if metric == "ip":
        base = base / np.linalg.norm(base, axis=1, keepdims=True)
    idx = build_index(base, 16, 8, iters=4, seed=3, metric=metric)
    h = amp.amp_index_from_arrays(idx)
    TQ = make_queries(w, 12, train=True)
    if metric == "ip":
        TQ = TQ / np.linalg.norm(TQ, axis=1, keepdims=True)
    TQ = TQ.astype(np.float32)
    rep = amp.amp_index_train_predictor(h, TQ, 10, 4, n_samples=40)
    assert rep["label_hist"] == _labels_by_definition(idx, TQ, 10, 4)
    assert rep["n_pairs"] == 12 * 4


def test_trainer_granularity_bounds_with_the_matching_quantiser():
    """Labels bound the error of the quantiser the search will use: with a
    width per (pair, subspace) the shift is never larger than with one width
    per pair by more than one step, so the labels are no wider on the whole."""
    w = WORKLOADS["mid"].scaled(n=40_000, nlist=64)
    base = make_base(w)
    idx = build_index(base, w.nlist, w.M, iters=5, seed=w.seed, integer_data=True)
    h = amp.amp_index_from_arrays(idx)
    TQ = make_queries(w, 48, train=True)
    rp = amp.amp_index_train_predictor(h, TQ, 10, 8, n_samples=200)
    rs = amp.amp_index_train_predictor(h, TQ, 10, 8, n_samples=200, granularity="subspace")
    assert rp["n_pairs"] == rs["n_pairs"]
    mean = lambda hist: sum(c * b for c, b in zip(hist, (4, 8, 12, 16))) / sum(hist)  # noqa: E731
    assert mean(rs["label_hist"]) <= mean(rp["label_hist"])
