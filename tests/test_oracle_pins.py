"""Pins of the CPU oracle against closed forms, brute force, library routines,
hand-worked fixtures and invariants (no GPU).  Each test names what it pins."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from amp_data import build_index, lossless_index, random_model, rbf_table
from amp_data.model import gamma_to_gmul
from amp_data.synth import WORKLOADS, make_base, make_queries

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ----------------------------------------------------------------- CL
def test_coarse_l2_and_ip_match_python_loops():
    r = np.random.default_rng(1)
    Q = r.normal(size=(3, 5)).astype(np.float32)
    C = r.normal(size=(7, 5)).astype(np.float32)
    for q in Q:
        D = oracle.coarse_distances(q, C, "l2")
        Dip = oracle.coarse_distances(q, C, "ip")
        for c in range(7):
            s = 0.0
            t = 0.0
            for j in range(5):
                s += (float(q[j]) - float(C[c, j])) ** 2
                t -= float(q[j]) * float(C[c, j])
            assert abs(D[c] - s) <= 1e-12 * max(1.0, s)
            assert abs(Dip[c] - t) <= 1e-12 * max(1.0, abs(t))


def test_coarse_l1_matches_python_loops():
    r = np.random.default_rng(21)
    Q = r.normal(size=(3, 6)).astype(np.float32)
    C = r.normal(size=(5, 6)).astype(np.float32)
    for q in Q:
        D = oracle.coarse_distances(q, C, "l1")
        for c in range(5):
            s = sum(abs(float(q[j]) - float(C[c, j])) for j in range(6))
            assert abs(D[c] - s) <= 1e-12 * max(1.0, s)


def test_select_probes_orders_by_distance_then_list_id():
    D = np.array([5.0, 1.0, 3.0, 1.0, 3.0, 0.5, 9.0])
    want = [c for _, c in sorted((float(D[c]), c) for c in range(len(D)))]
    assert oracle.select_probes(D, 7).tolist() == want
    assert oracle.select_probes(D, 3).tolist() == [5, 1, 3]


# ----------------------------------------------------------------- RC
def test_residual_is_correctly_rounded_fp32_subtraction():
    r = np.random.default_rng(2)
    a = (r.normal(size=4000) * 10.0 ** r.integers(-8, 8, size=4000)).astype(np.float32)
    b = (r.normal(size=4000) * 10.0 ** r.integers(-8, 8, size=4000)).astype(np.float32)
    a[:4] = [1.0, 3.0e38, 1e-30, 16777216.0]
    b[:4] = [np.float32(1.0) - np.float32(2.0 ** -24), -3.0e38, 1e-38, 1.0]
    with np.errstate(over="ignore"):
        want = a - b  # IEEE float32 subtraction (round to nearest even)
        got = np.array([oracle.residual_f32(x, y) for x, y in zip(a, b)], dtype=np.float32)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_u9_grid_rounds_half_even_and_saturates():
    x = np.array([0.5, 1.5, 2.5, -0.5, -1.5, 254.5, 255.5, 300.0, -300.0, 7.49999, -7.5])
    want = [0, 2, 2, 0, -2, 254, 255, 255, -255, 7, -8]
    assert oracle.grid(x, "u9").tolist() == want


def _e4m3_values_from_spec():
    """Decode all E4M3 (OCP 8-bit float, 'fn' variant) bit patterns: bias 7,
    subnormals m/8 * 2^-6, S.1111.111 is NaN, no infinities."""
    vals = []
    for e in range(16):
        for m in range(8):
            if e == 15 and m == 7:
                continue
            v = Fraction(m, 8) * Fraction(1, 64) if e == 0 else (1 + Fraction(m, 8)) * Fraction(2) ** (e - 7)
            vals.append((v, m))
    return vals


def test_e4m3_integer_rounding_matches_spec_table():
    vals = _e4m3_values_from_spec()
    for x in range(-700, 701):
        a = abs(x)
        if a >= 464:            # at or above the midpoint 448..480: saturate
            want = 448
        else:
            best = min(vals, key=lambda vm: (abs(vm[0] - a), vm[1] % 2))
            want = best[0]
        got = int(oracle.e4m3_round_int(np.array([x]))[0])
        assert Fraction(got) == (want if x >= 0 else -want), x


def test_e4m3_rounding_agrees_with_torch_cast():
    torch = pytest.importorskip("torch")
    if not hasattr(torch, "float8_e4m3fn"):
        pytest.skip("torch without float8_e4m3fn")
    x = np.arange(-460, 461)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.float8_e4m3fn).to(torch.float32).numpy()
    got = oracle.e4m3_round_int(x)
    assert np.array_equal(got, ref.astype(np.int64))


# ----------------------------------------------------------------- LC
def test_lut_int_identity_sum_equals_direct_distance():
    """I1: sum_m T[m][code_m] = ||ri - cbi(code)||^2 (exact integers)."""
    r = np.random.default_rng(3)
    M, dsub = 6, 4
    cbi = r.integers(-255, 256, size=(M, 256, dsub))
    ri = r.integers(-255, 256, size=M * dsub)
    T = oracle.lut_int(ri, cbi, "l2")
    Tip = oracle.lut_int(ri, cbi, "ip")
    for _ in range(50):
        code = r.integers(0, 256, size=M)
        rec = [int(v) for m in range(M) for v in cbi[m, code[m]]]
        direct = sum((int(a) - b) ** 2 for a, b in zip(ri, rec))
        assert int(sum(T[m, code[m]] for m in range(M))) == direct
        assert int(sum(Tip[m, code[m]] for m in range(M))) == -sum(int(a) * b for a, b in zip(ri, rec))


def test_l1_lut_sum_equals_direct_distance():
    """L1 is separable over coordinates: sum_m T[m][code_m] = |ri - cbi(code)|_1
    (exact integers), and the FP64 LUT of the FP32 residual sums to the L1
    distance from the query to the reconstruction."""
    r = np.random.default_rng(22)
    M, dsub = 5, 4
    cbi = r.integers(-255, 256, size=(M, 256, dsub))
    ri = r.integers(-255, 256, size=M * dsub)
    T = oracle.lut_int(ri, cbi, "l1")
    CB = r.normal(size=(M, 256, dsub)).astype(np.float32)
    c = r.normal(size=M * dsub).astype(np.float32) * 3
    q = r.normal(size=M * dsub).astype(np.float32) * 3
    res = oracle.residual_f32(q, c)
    T64 = oracle.lut_f64(res, CB, "l1")
    for _ in range(40):
        code = r.integers(0, 256, size=M)
        rec = [int(v) for m in range(M) for v in cbi[m, code[m]]]
        assert int(sum(T[m, code[m]] for m in range(M))) == sum(abs(int(a) - b) for a, b in zip(ri, rec))
        xr = np.concatenate([CB[m, code[m]] for m in range(M)]).astype(np.float64)
        direct = float(np.abs(res.astype(np.float64) - xr).sum())
        assert abs(float(sum(T64[m, code[m]] for m in range(M))) - direct) <= 1e-12 * direct


def test_full_precision_adc_equals_reconstruction_distance():
    """Full-precision ADC sum = ||q - x_hat||^2, x_hat = c + concat cb(code)."""
    r = np.random.default_rng(4)
    M, dsub, d = 8, 4, 32
    CB = r.normal(size=(M, 256, dsub)).astype(np.float32)
    c = r.normal(size=d).astype(np.float32) * 5
    for _ in range(20):
        q = r.normal(size=d).astype(np.float32) * 5
        code = r.integers(0, 256, size=M)
        res = oracle.residual_f32(q, c)
        T = oracle.lut_f64(res, CB)
        adc = float(sum(T[m, code[m]] for m in range(M)))
        xhat = c.astype(np.float64) + np.concatenate([CB[m, code[m]] for m in range(M)]).astype(np.float64)
        direct = float(((res.astype(np.float64) + c - xhat) ** 2).sum())
        assert abs(adc - direct) <= 1e-12 * direct


# ----------------------------------------------------------------- quantiser
def test_quantizer_hand_worked_fixture():
    g = _gold("quantize_worked.json")
    T = np.array(g["T"])
    for case in g["cases"]:
        Q, s, base = oracle.quantize_lut(T, case["b"])
        assert s == case["s"] and base == case["base"]
        assert Q.tolist() == case["Q"]
        for codes, est, ex in zip(case["codes"], case["estimate"], case["exact"]):
            S = sum(int(Q[m, c]) for m, c in enumerate(codes))
            assert base + (S << s) == est
            assert sum(int(T[m, c]) for m, c in enumerate(codes)) == ex


@pytest.mark.parametrize("b", [4, 8, 12, 16])
def test_quantizer_bounds_and_rounding(b):
    """I2 range, I3 error bound, I4 exact case, minimal shift, and the rounding
    checked with exact rationals."""
    r = np.random.default_rng(10 + b)
    for trial in range(30):
        M = int(r.integers(1, 9))
        scale = int(10 ** r.integers(1, 7))
        T = r.integers(0, scale, size=(M, 256)) + r.integers(-1000, 1000, size=(M, 1))
        Q, s, base = oracle.quantize_lut(T, b)
        top = (1 << b) - 1
        assert Q.min() >= 0 and Q.max() <= top                         # I2
        lo = T.min(1)
        R = int((T - lo[:, None]).max())
        hf = lambda t: (1 << (t - 1)) if t else 0  # noqa: E731
        assert ((R + hf(s)) >> s) <= top
        if s > 0:
            assert ((R + hf(s - 1)) >> (s - 1)) > top                    # minimal s
        else:
            assert R <= top                                              # I4
        for m in range(M):
            for j in r.integers(0, 256, size=8):
                exact = Fraction(int(T[m, j] - lo[m]), 1 << s)
                assert int(Q[m, j]) == math.floor(exact + Fraction(1, 2))
        codes = r.integers(0, 256, size=(40, M))
        for cd in codes:
            Dint = sum(int(T[m, cd[m]]) for m in range(M))
            Dq = base + (sum(int(Q[m, cd[m]]) for m in range(M)) << s)
            assert abs(Dq - Dint) <= M * (hf(s))                       # I3
            if s == 0:
                assert Dq == Dint


# ----------------------------------------------------------------- PPM
def test_mitchell_log2_hand_worked_and_bounds():
    g = _gold("mitchell_log2.json")
    assert oracle.mitchell_log2_q8(np.array(g["x"])).tolist() == g["L"]
    x = np.concatenate([np.arange(0, 5000), (2 ** np.arange(0, 40)) - 1,
                        np.random.default_rng(5).integers(0, 2 ** 40, size=2000)])
    L = oracle.mitchell_log2_q8(x)
    # exact at powers of two, within Mitchell's maximum error (0.0861) elsewhere
    pw = (2 ** np.arange(0, 40)) - 1
    assert oracle.mitchell_log2_q8(pw).tolist() == (256 * np.arange(0, 40)).tolist()
    err = np.abs(L / 256.0 - np.log2(x.astype(np.float64) + 1))
    assert err.max() <= 0.0861 + 1 / 256
    xs = np.sort(x)
    assert np.all(np.diff(oracle.mitchell_log2_q8(xs)) >= 0)


def _worked_model(g):
    m = dict(g["model"])
    assert m.pop("table_rule") == "1024 - i"
    m["table"] = np.array([1024 - i for i in range(1024)], dtype=np.int64)
    m["sv"] = np.asarray(m["sv"], dtype=np.int64)
    m["beta"] = np.asarray(m["beta"], dtype=np.int64)
    m["n_sv"] = len(m["beta"])
    return m


def test_predictor_hand_worked_fixture():
    """Features, C1 choice, affine map with clamps, table-read RBF score and
    width choice (thresholds inclusive, margin, allowed sets with and without
    12 bits) against the hand-worked values of tests/golden/predictor_worked.json."""
    g = _gold("predictor_worked.json")
    m = _worked_model(g)
    for x, L in g["log2_q8"].items():
        assert int(oracle.mitchell_log2_q8(np.array([int(x)]))[0]) == L
    P = np.asarray(g["probes"])
    dq2 = np.asarray(g["dq2"])
    radq, sizes = np.asarray(g["radq"]), np.asarray(g["sizes"])
    c1 = g["c1"]
    for i, p in enumerate(P.tolist()):
        x = [int(dq2[i]), int(radq[c1]), int(radq[p]), int(sizes[c1]), int(sizes[p])]
        u = oracle.feature_u(x, m)
        assert u.tolist() == g["u"][i]
        assert oracle.svr_eval(u, m) == g["score"][i]
    for case in g["cases"]:
        bits, ys = oracle.predict_pair_bits(dq2, P, radq, sizes, m, case["allowed"], case["margin"])
        assert bits.tolist() == case["bits"], case
        assert [int(y) for y in ys] == g["score"]


def _lin_model(n_sv=64, gamma=1.0, seed=0):
    return random_model(seed, n_sv, feat_lo=[0] * 5, feat_mul=[1 << 12] * 5, gamma=gamma)


def test_rbf_kernel_table_matches_gaussian_within_table_step():
    """The table-read kernel equals exp(-gamma ||du/1023||^2) within the
    table's resolution (1/64 in the exponent, Q20 values)."""
    for gamma in (0.1, 1.0, 3.0):
        m = _lin_model(gamma=gamma)
        table = np.asarray(m["table"], dtype=np.float64) / 2 ** 20
        r = np.random.default_rng(6)
        for _ in range(200):
            du = r.integers(-1023, 1024, size=5)
            dist2 = int((du * du).sum())
            idx = min((dist2 * m["g_mul"]) >> 32, 1023)
            arg = gamma * dist2 / 1023 ** 2
            if arg * 64 >= 1023:
                continue
            # table midpoint rule: |exp(-a) - exp(-(i+1/2)/64)| <= exp(-a)(e^(1/128)-1) + rounding
            tol = math.exp(-arg) * (math.exp(1 / 128 + 1e-6) - 1) + 2 ** -20 + 1e-9
            assert abs(table[idx] - math.exp(-arg)) <= tol * 1.01 + abs(
                gamma_to_gmul(gamma) / 2 ** 32 - gamma * 64 / 1023 ** 2) * dist2 * math.exp(-arg)


def test_svr_score_matches_real_rbf_regression():
    """y / 2^40 = beta0 + sum beta_i exp(-gamma ||u - s_i||^2) within the
    table error; the regressor sums over every support vector."""
    m = _lin_model(n_sv=100, gamma=1.0, seed=3)
    r = np.random.default_rng(7)
    for _ in range(30):
        u = r.integers(0, 1024, size=5)
        y = oracle.svr_eval(u, m) / 2.0 ** 40
        du = (np.asarray(m["sv"], dtype=np.float64) - u) / 1023.0
        K = np.exp(-1.0 * (du * du).sum(1))
        beta = np.asarray(m["beta"], dtype=np.float64) / 2 ** 20
        ref = m["beta0"] / 2.0 ** 40 + float((beta * K).sum())
        bound = float(np.abs(beta).sum()) * (math.exp(1 / 128) - 1 + 2 ** -19)
        assert abs(y - ref) <= bound


def test_degenerate_predictor_gives_constant_bits_and_thresholds_are_inclusive():
    m = _lin_model()
    m["beta"] = np.zeros_like(m["beta"])
    for b0, want in [(-0.5, 4), (-0.2, 4), (-0.1, 8), (0.0, 8), (0.1, 12), (0.3, 16)]:
        m["beta0"] = int(round(b0 * 2 ** 40))
        u = np.random.default_rng(8).integers(0, 1024, size=5)
        y = oracle.svr_eval(u, m)
        assert y == m["beta0"]
        assert oracle.bits_from_score(y, m) == want
    # allowed subsets: never returns a disallowed width
    m["beta0"] = int(0.1 * 2 ** 40)
    assert oracle.bits_from_score(m["beta0"], m, allowed=(4, 8, 16)) == 16
    assert oracle.bits_from_score(m["beta0"], m, allowed=(4, 8)) == 8
    m["beta0"] = int(-0.5 * 2 ** 40)
    assert oracle.bits_from_score(m["beta0"], m, allowed=(8, 16)) == 8


def test_single_support_vector_score_decreases_with_distance():
    m = _lin_model(n_sv=1)
    m["sv"] = np.array([[500] * 5], dtype=np.int32)
    m["beta"] = np.array([1 << 20], dtype=np.int32)
    m["beta0"] = 0
    ys = [oracle.svr_eval(np.array([500 + t] * 5), m) for t in range(0, 500, 25)]
    assert all(a >= b for a, b in zip(ys, ys[1:])) and ys[0] > ys[-1]


# ----------------------------------------------------------------- DC + TS
def _tiny_index(seed=11, n=3000, d=16, nlist=12, M=4):
    r = np.random.default_rng(seed)
    means = r.uniform(-5, 5, size=(nlist, d))
    base = (means[r.integers(0, nlist, size=n)] + r.normal(size=(n, d))).astype(np.float32)
    idx = build_index(base, nlist, M, iters=8, seed=seed)
    return idx, base


def test_search_equals_bruteforce_over_all_candidates():
    idx, base = _tiny_index()
    Q = np.random.default_rng(12).normal(size=(6, 16)).astype(np.float32) * 3
    for policy, b in [("fixed", 4), ("fixed", 8), ("fixed", 16)]:
        res = oracle.search(idx, Q, k=7, nprobe=5, policy=policy, bits=b)
        cbi, _ = oracle.index_grid(idx)
        for i, q in enumerate(Q):
            D = oracle.coarse_distances(q, idx["centroids"])
            P = sorted(range(idx["nlist"]), key=lambda c: (D[c], c))[:5]
            assert res["probes"][i].tolist() == P
            cands = []
            for p in P:
                rr = oracle.grid(oracle.residual_f32(q, idx["centroids"][p]).astype(np.float64)
                                 * 2.0 ** -idx["grid_e"])
                Qt, s, base0 = oracle.quantize_lut(oracle.lut_int(rr, cbi), b)
                for pos in range(idx["list_offsets"][p], idx["list_offsets"][p + 1]):
                    S = sum(int(Qt[m, idx["codes"][pos, m]]) for m in range(idx["M"]))
                    cands.append((base0 + (S << s), int(idx["ids"][pos])))
            cands.sort()
            assert res["ids"][i].tolist() == [c[1] for c in cands[:7]]
            assert res["qdist"][i].tolist() == [c[0] for c in cands[:7]]
            assert len({c[1] for c in cands}) == len(cands)


def test_padding_when_fewer_candidates_than_k():
    idx, _ = _tiny_index(n=60, nlist=12)
    q = np.zeros((1, 16), dtype=np.float32)
    res = oracle.search(idx, q, k=50, nprobe=1, policy="fixed", bits=16)
    p = res["probes"][0, 0]
    n = int(idx["list_sizes"][p])
    assert n < 50
    assert (res["ids"][0, n:] == -1).all()
    assert (res["qdist"][0, n:] == np.iinfo(np.int64).max).all()
    assert np.isinf(res["dist"][0, n:]).all()


def test_lossless_index_recovers_exact_knn():
    """Base vectors are exactly centroid + codewords: with every list probed,
    the full-precision search and the exact integer search (s = 0) return the
    exact k nearest neighbours with their exact distances."""
    idx, base = lossless_index(seed=5, nlist=6, M=4, dsub=4, per_list=[40, 3, 77, 0, 12, 60])
    Q = np.random.default_rng(13).integers(-40, 41, size=(8, 16)).astype(np.float32)
    truth = oracle.exact_knn(base, Q, 10)
    r32 = oracle.search(idx, Q, 10, 6, policy="fp32")
    assert np.array_equal(r32["ids"], truth)
    r16 = oracle.search(idx, Q, 10, 6, policy="fixed", bits=16)
    assert (r16["shift"] == 0).all()
    assert np.array_equal(r16["ids"], truth)
    d64 = ((base[truth].astype(np.float64) - Q[:, None, :]) ** 2).sum(-1)
    assert np.array_equal(r16["qdist"], d64.astype(np.int64))
    assert oracle.recall_at(r16["ids"], truth) == 1.0


def test_lossless_index_recovers_exact_l1_knn():
    """Special case for the L1 mode: integer queries, base vectors exactly
    centroid + codewords, every list probed: the exact integer search (s = 0)
    returns the exact L1 nearest neighbours with their exact distances."""
    idx, base = lossless_index(seed=5, nlist=6, M=4, dsub=4, per_list=[40, 3, 77, 0, 12, 60])
    idx = dict(idx, metric="l1")
    Q = np.random.default_rng(14).integers(-40, 41, size=(8, 16)).astype(np.float32)
    truth = oracle.exact_knn(base, Q, 10, "l1")
    r16 = oracle.search(idx, Q, 10, 6, policy="fixed", bits=16)
    assert (r16["shift"] == 0).all()
    assert np.array_equal(r16["ids"], truth)
    d1 = np.abs(base[truth].astype(np.float64) - Q[:, None, :]).sum(-1)
    assert np.array_equal(r16["qdist"], d1.astype(np.int64))
    r32 = oracle.search(idx, Q, 10, 6, policy="fp32")
    assert np.array_equal(r32["ids"], truth)


def test_lossless_index_recovers_exact_inner_product_knn():
    """Special case for the inner-product metric: integer queries, base
    vectors exactly centroid + codewords, every list probed at 16 bits: the
    integer estimate is -<q, x> exactly (s = 0) and the ids are the exact
    inner-product neighbours; the full-precision policy returns the same ids."""
    idx, base = lossless_index(seed=9, nlist=6, M=4, dsub=4, per_list=[40, 3, 77, 0, 12, 60])
    idx = dict(idx, metric="ip")
    Q = np.random.default_rng(15).integers(-40, 41, size=(8, 16)).astype(np.float32)
    truth = oracle.exact_knn(base, Q, 10, "ip")
    r16 = oracle.search(idx, Q, 10, 6, policy="fixed", bits=16)
    assert (r16["shift"] == 0).all()
    assert np.array_equal(r16["ids"], truth)
    ip = (base[truth].astype(np.float64) * Q[:, None, :]).sum(-1)
    assert np.array_equal(r16["qdist"], -ip.astype(np.int64))
    r32 = oracle.search(idx, Q, 10, 6, policy="fp32")
    assert np.array_equal(r32["ids"], truth)
    assert np.array_equal(r32["dist"], (-ip).astype(np.float32))


def test_full_precision_inner_product_adc_equals_reconstruction_score():
    """Inner product: the full-precision LUT sum plus the list term -<q, c> is
    -<q, x_hat> with x_hat = c + concat cb(code), to FP64 rounding."""
    r = np.random.default_rng(16)
    M, dsub, d = 8, 4, 32
    CB = r.normal(size=(M, 256, dsub)).astype(np.float32)
    c = r.normal(size=d).astype(np.float32) * 5
    for _ in range(20):
        q = r.normal(size=d).astype(np.float32) * 5
        code = r.integers(0, 256, size=M)
        T = oracle.lut_f64(q, CB, "ip")
        add = -float(q.astype(np.float64) @ c.astype(np.float64))
        adc = add + float(sum(T[m, code[m]] for m in range(M)))
        xhat = c.astype(np.float64) + np.concatenate([CB[m, code[m]] for m in range(M)]).astype(np.float64)
        direct = -float(q.astype(np.float64) @ xhat)
        scale = float(np.abs(q.astype(np.float64)) @ np.abs(xhat))
        assert abs(adc - direct) <= 1e-12 * scale


@pytest.mark.parametrize("e", [1, -1])
def test_lossless_index_on_a_power_of_two_grid_step(e):
    """index_grid and the grid exponent: centroids, codewords and queries are
    multiples of h = 2^e, so every residual and codeword maps to the grid
    exactly; the 16-bit search then returns the exact neighbours with integer
    estimates D / h^2 and reported distances D (L2 and inner product)."""
    h = 2.0 ** e
    idx0, base0 = lossless_index(seed=6, nlist=5, M=4, dsub=4, per_list=[30, 8, 0, 50, 21],
                                 cb_range=6, c_range=30)
    idx = dict(idx0, grid_e=e, centroids=(idx0["centroids"] * h).astype(np.float32),
               codebook=(idx0["codebook"] * h).astype(np.float32))
    base = (base0 * h).astype(np.float32)
    cbi, ci = oracle.index_grid(idx)
    assert np.array_equal(cbi, idx0["codebook"].astype(np.int64))
    assert np.array_equal(ci, idx0["centroids"].astype(np.int64))
    Q = (np.random.default_rng(17).integers(-30, 31, size=(6, 16)) * h).astype(np.float32)
    for metric in ("l2", "ip"):
        im = dict(idx, metric=metric)
        truth = oracle.exact_knn(base, Q, 8, metric)
        res = oracle.search(im, Q, 8, 5, policy="fixed", bits=16)
        assert (res["shift"] == 0).all()
        assert np.array_equal(res["ids"], truth)
        X = base[truth].astype(np.float64)
        D = ((X - Q[:, None, :]) ** 2).sum(-1) if metric == "l2" else -(X * Q[:, None, :]).sum(-1)
        assert np.array_equal(res["qdist"].astype(np.float64) * h * h, D)
        assert np.array_equal(res["dist"], D.astype(np.float32))


@pytest.mark.parametrize("metric", ["l2", "ip", "l1"])
def test_exact_knn_matches_a_python_sort_with_ties(metric):
    """Brute force: exact_knn equals Python's sort of (distance, id) over every
    vector, with duplicated vectors so that ties must go to the lower id."""
    r = np.random.default_rng(18)
    B = r.integers(-3, 4, size=(60, 5)).astype(np.float32)
    B[30:45] = B[0:15]  # exact duplicates: equal distances at different ids
    Q = r.integers(-3, 4, size=(7, 5)).astype(np.float32)
    got = oracle.exact_knn(B, Q, 12, metric)
    for i, q in enumerate(Q):
        def dist(x):
            if metric == "l2":
                return sum((float(a) - float(b)) ** 2 for a, b in zip(x, q))
            if metric == "l1":
                return sum(abs(float(a) - float(b)) for a, b in zip(x, q))
            return -sum(float(a) * float(b) for a, b in zip(x, q))
        want = [j for _, j in sorted((dist(B[j]), j) for j in range(len(B)))][:12]
        assert got[i].tolist() == want
    assert oracle.exact_knn(B[:5], Q[:2], 8, metric)[:, 5:].tolist() == [[-1] * 3] * 2


@pytest.mark.slow
def test_tiny_workload_recall_against_exact_knn():
    w = WORKLOADS["tiny"].scaled(n=20_000, nq=40)
    base = make_base(w)
    idx = build_index(base, w.nlist, w.M, iters=10, seed=w.seed)
    Q = make_queries(w, 40)
    truth = oracle.exact_knn(base, Q, 10)
    rec = {}
    for npb in (1, 8, 64):
        res = oracle.search(idx, Q, 10, npb, policy="fixed", bits=16)
        rec[npb] = oracle.recall_at(res["ids"], truth)
    r32 = oracle.recall_at(oracle.search(idx, Q, 10, 8, policy="fp32")["ids"], truth)
    assert rec[1] <= rec[8] <= rec[64] + 1e-9
    assert rec[8] >= 0.3 and abs(rec[8] - r32) <= 0.05


# ------------------------------------------------- quantiser: per-subspace widths
def test_subspace_granularity_hand_worked():
    """Two subspaces with ranges 10 and 100, b = 4.  One width per pair: the
    largest range sets s = 3 ((100 + 4) >> 3 = 13 <= 15, (100 + 2) >> 2 = 25
    > 15).  Per-subspace widths: the budget 2 * 15 = 30 for the sum 110 gives
    s = 2 ((110 + 2 * 2) >> 2 = 28 <= 30, (110 + 2 * 1) >> 1 = 56 > 30); the
    first subspace then uses entries up to (10 + 2) >> 2 = 3 (2 bits), the
    second up to (100 + 2) >> 2 = 25 (5 bits)."""
    T = np.zeros((2, 256), np.int64)
    T[0, :11] = np.arange(11) + 7        # range 10, minimum 7
    T[0, 11:] = 12
    T[1, :101] = np.arange(101) - 40     # range 100, minimum -40
    T[1, 101:] = 0
    Q, s, base = oracle.quantize_lut(T, 4)
    assert s == 3 and base == 7 - 40 and Q.max() == 13
    Q, s, base = oracle.quantize_lut(T, 4, "subspace")
    assert s == 2 and base == -33
    assert Q[0].max() == 3 and Q[1].max() == 25
    # entry (m = 1, j = 57): T = 17, (17 + 40 + 2) >> 2 = 14
    assert Q[1, 57] == 14


@pytest.mark.parametrize("b", [4, 8, 12, 16])
def test_subspace_granularity_budget_and_error(b):
    """Any vector's sum of entries fits the pair's lane budget M (2^b - 1);
    the estimate is within M 2^(s-1) of the exact sum (round half up: each
    entry within (-2^(s-1), 2^(s-1)] of its exact value); the shift is the
    smallest with the budget, checked by brute force over all codes' maxima."""
    r = np.random.default_rng(40 + b)
    for trial in range(30):
        M = int(r.integers(1, 17))
        scales = 10 ** r.integers(1, 7, size=M)
        T = np.stack([r.integers(0, int(sc), size=256) for sc in scales]) + r.integers(-999, 999, size=(M, 1))
        Q, s, base = oracle.quantize_lut(T, b, "subspace")
        top = M * ((1 << b) - 1)
        assert int(Q.max(1).sum()) <= top                      # the lane never overflows
        lo = T.min(1)
        if s > 0:
            # one shift less would exceed the budget for the range sum
            R = int((T - lo[:, None]).max(1).sum())
            hf = (1 << (s - 2)) if s > 1 else 0
            assert (R + M * hf) >> (s - 1) > top
        codes = r.integers(0, 256, size=(200, M))
        est = base + (Q[np.arange(M)[None, :], codes].sum(1) << s)
        ex = T[np.arange(M)[None, :], codes].sum(1)
        half = (1 << (s - 1)) if s else 0
        assert np.all(np.abs(est - ex) <= M * max(half, 0))
        if s == 0:
            assert np.array_equal(est, ex)
        # per subspace the estimate error of an entry is within (-half, half]
        err = (Q << s) - (T - lo[:, None])
        assert err.max() <= half and (s == 0 or err.min() > -half)


def test_subspace_granularity_is_as_fine_for_equal_ranges():
    """With equal ranges the per-subspace rule is the per-pair rule up to the
    rounding of the shared half-unit: never coarser by more than one step."""
    r = np.random.default_rng(7)
    for _ in range(50):
        M, b = int(r.integers(2, 17)), int(r.choice([4, 8, 12, 16]))
        R = int(r.integers(1, 10 ** 6))
        T = np.zeros((M, 256), np.int64)
        T[:, 1] = R
        s_pair = oracle.quantize_lut(T, b)[1]
        s_sub = oracle.quantize_lut(T, b, "subspace")[1]
        assert s_sub <= s_pair + 1
