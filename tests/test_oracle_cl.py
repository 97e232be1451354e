"""Pins of the oracle's reduced-precision cluster locating (oracle/cl.py):
hand-worked values, brute force and closed forms, independent of the
functions under test."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import cl as ocl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold():
    with open(os.path.join(GOLD, "cl_worked.json")) as f:
        return json.load(f)


def _map(g):
    return dict(S=g["S"], P=g["P"], centre=np.array(g["centre"]), radius=np.array(g["radius"]),
                count=np.array(g["count"]), assign=np.array(g["assign"]), o=np.float32(0), ec=0)


def test_trunc_is_floor_to_a_multiple_of_the_dropped_bits():
    # every 8-bit code and width, against Python's integer floor division
    for b in range(1, 9):
        step = 2 ** (8 - b)
        v = np.arange(-128, 128)
        want = np.array([(int(x) // step) * step for x in v])
        assert np.array_equal(ocl.trunc(v, b), want), b
    assert np.array_equal(ocl.trunc(np.arange(-128, 128), 8), np.arange(-128, 128))
    # two's-complement view: the top b bits of the byte
    for x in (-20, -1, -128, 127, 37):
        assert int(ocl.trunc(x, 4)) == int(np.int8(np.uint8(np.int8(x).view(np.uint8) & 0xF0).view(np.int8)))


def test_codes_round_half_to_even_and_clamp():
    o, ec = np.float32(0.5), 1
    x = np.array([3.5, 5.5, -2.5, 0.5, 1.5, 1000.0, -1000.0, 255.0, -255.0], dtype=np.float32)
    # (x - o) / 2 = 1.5, 2.5, -1.5, 0, 0.5, 499.75, -500.25, 127.25, -127.75
    assert ocl.cl_codes(x, o, ec).tolist() == [2, 2, -2, 0, 0, 127, -128, 127, -128]


def test_code_parameters():
    C = np.array([[0.0, 200.0], [50.0, 120.0]], np.float32)
    assert ocl.cl_params(C, "l2") == (np.float32(100.0), 0)  # half-range 100 <= 127
    C = np.array([[-3.0, 1000.0]], np.float32)
    o, ec = ocl.cl_params(C, "l2")
    assert o == np.float32(498.5) and ec == 2  # 501.5 > 254, <= 508
    C = np.array([[-0.3, 0.25]], np.float32)
    o, ec = ocl.cl_params(C, "ip")
    assert o == 0 and ec == -8  # 0.3 > 127/512 = 0.248, <= 127/256 = 0.496
    # every centroid code of a random set is within [-127, 127] before clamping
    r = np.random.default_rng(5)
    C = r.normal(3.0, 40.0, size=(50, 16)).astype(np.float32)
    o, ec = ocl.cl_params(C, "l2")
    raw = np.rint((C.astype(np.float32) - o).astype(np.float64) * 2.0 ** -ec)
    assert np.abs(raw).max() <= 127 and np.abs(raw).max() > 63


def test_full_width_equals_the_exact_distance_of_integer_data():
    # integer data with an integer offset: codes are exact shifts, so the
    # 8-bit CL distance is the exact distance of the original vectors
    r = np.random.default_rng(11)
    d, S = 12, 3
    X = r.integers(0, 255, size=(40, d)).astype(np.float32)
    X[0, 0], X[1, 1] = 0, 254
    o, ec = ocl.cl_params(X, "l2")
    assert o == 127 and ec == 0
    q = r.integers(0, 255, size=d).astype(np.float32)
    assign = r.integers(0, 4, size=(40, S))
    bits = np.full((S, 4), 8)
    D = ocl.coarse_mixed(ocl.cl_codes(q, o, ec), ocl.cl_codes(X, o, ec), assign, bits, S, "l2")
    want = [sum((int(a) - int(b)) ** 2 for a, b in zip(q, x)) for x in X]
    assert D.tolist() == want
    # inner product, offset 0
    Y = r.integers(-100, 101, size=(40, d)).astype(np.float32)
    oy, ey = ocl.cl_params(Y, "ip")
    assert oy == 0 and ey == 0
    qy = r.integers(-100, 101, size=d).astype(np.float32)
    D = ocl.coarse_mixed(ocl.cl_codes(qy, oy, ey), ocl.cl_codes(Y, oy, ey), assign, bits, S, "ip")
    assert D.tolist() == [-sum(int(a) * int(b) for a, b in zip(qy, y)) for y in Y]


def test_hand_worked_mixed_width_distances_and_probes():
    g = _gold()
    m = _map(g)
    q, Vc = np.array(g["q"]), np.array(g["Vc"])
    D = ocl.coarse_mixed(q, Vc, m["assign"], np.array(g["bits"]), 2, "l2")
    assert D.tolist() == g["D_l2"]
    Df = ocl.coarse_mixed(q, Vc, m["assign"], np.full((2, 2), 8), 2, "l2")
    assert Df.tolist() == g["D_l2_full"]
    assert oracle.select_probes(D, 2).tolist() == g["probes2_mixed"]
    assert oracle.select_probes(Df, 2).tolist() == g["probes2_full"]
    assert ocl.coarse_mixed(q, Vc, m["assign"], np.array(g["bits"]), 2, "ip").tolist() == g["D_ip"]


def test_hand_worked_features_and_c1_ties():
    g = _gold()
    m = _map(g)
    d2, c1 = ocl.subspace_features(np.array(g["q"]), m)
    assert d2.tolist() == g["d2"] and c1.tolist() == g["c1"]
    d2, c1 = ocl.subspace_features(np.array(g["q2"]), m)
    assert d2.tolist() == g["q2_d2"] and c1.tolist() == g["q2_c1"]  # slice 0: tie -> lower index


def test_prediction_scores_the_hand_worked_feature_vectors():
    """predict_cl_bits assembles [d', r1, r2, n1, n2] as worked by hand and
    applies the threshold inclusively (the regressor itself is pinned by the
    LUT predictor's worked example)."""
    g = _gold()
    m = _map(g)
    model = dict(sv=np.array([[0, 300, 100, 500, 0], [800, 0, 900, 0, 1000]]), beta=np.array([5, -3]), beta0=10,
                 table=np.arange(1024, 0, -1), g_mul=1 << 22, feat_lo=np.array([1000, 0, 0, 0, 0]),
                 feat_mul=np.array([40000, 65536, 65536, 65536, 65536]), theta=np.array([0, 0, 0]))
    want = np.array([[oracle.svr_eval(oracle.feature_u(x, model), model) for x in row] for row in g["x5"]])
    bits, ys = ocl.predict_cl_bits(np.array(g["q"]), m, model, 4)
    assert ys.astype(np.int64).tolist() == want.tolist()
    for th in (int(want.min()), int(np.median(want)), int(want.max())):
        model["theta"] = np.array([th, 0, 0])
        bits, _ = ocl.predict_cl_bits(np.array(g["q"]), m, model, 3)
        assert bits.tolist() == np.where(want <= th, 3, 8).tolist()


def test_low_share_counts_partial_distances():
    g = _gold()
    m = _map(g)
    # widths [[4, 8], [8, 4]]: low partials = count[0][0] + count[1][1] = 2 + 2 of 6
    assert ocl.low_share(np.array(g["bits"]), m, 4) == pytest.approx(4 / 6)


def test_mixed_width_error_bound():
    """Each truncated coordinate moves a squared difference by at most
    2 |x| 2^k + 2^(2k) (k = 8 - b dropped bits, x the full-width difference):
    the sum of the bounds holds for random codes and widths."""
    r = np.random.default_rng(2)
    d, S, P = 24, 4, 3
    Vc = r.integers(-128, 128, size=(30, d))
    q = r.integers(-128, 128, size=d)
    assign = r.integers(0, P, size=(30, S))
    bits = r.choice([2, 4, 6, 8], size=(S, P))
    D = ocl.coarse_mixed(q, Vc, assign, bits, S, "l2")
    Df = ocl.coarse_mixed(q, Vc, assign, np.full((S, P), 8), S, "l2")
    for i in range(30):
        bound = 0
        for s, (a, b) in enumerate(ocl.slices(d, S)):
            k = 8 - int(bits[s, assign[i, s]])
            x = np.abs(q[a:b] - Vc[i, a:b])
            bound += int((2 * x * 2 ** k + 2 ** (2 * k)).sum()) if k else 0
        assert abs(int(D[i]) - int(Df[i])) <= bound
