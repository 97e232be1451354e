"""GPU autotuner (amp_index_autotune / amp_index_set_tuning): a search's
schedule (unit chunking, LUT row width, LC dtype, unit queue) changes how work is cut,
never the result; the tuner records the fastest schedule it timed."""
import numpy as np
import pytest

import paper_2606_07156_amd as amp
from amp_data import build_index
from amp_data.synth import WORKLOADS, make_base, make_queries

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mid():
    # the mid workload's shape (M = 16: wide LUT rows exist) at test size
    w = WORKLOADS["mid"].scaled(n=60_000, nq=96, nlist=128)
    idx = build_index(make_base(w), w.nlist, w.M, iters=6, seed=w.seed, integer_data=True)
    h = amp.amp_index_from_arrays(idx)
    amp.amp_index_to_device(h, 0)
    return dict(h=h, Q=make_queries(w, 96), idx=idx)


SCHEDULES = [
    dict(chunk=256, chunk1=0, narrow=-1, lut_dtype=0),
    dict(chunk=0, chunk1=256, narrow=1, lut_dtype=0),
    dict(chunk=512, chunk1=256, narrow=0, lut_dtype=0),
    dict(chunk=0, chunk1=0, narrow=0, lut_dtype=amp.AMP_LUT_F16),
    dict(chunk=1024, chunk1=0, narrow=1, lut_dtype=amp.AMP_LUT_F16),
    dict(chunk=0, chunk1=0, narrow=-1, lut_dtype=0, queue=1),
    dict(chunk=256, chunk1=256, narrow=1, lut_dtype=0, queue=1),
]


@pytest.mark.parametrize("policy,bits", [("fixed", 4), ("fixed", 12), ("fp32", 0)])
def test_every_schedule_returns_the_same_results(mid, policy, bits):
    kind = amp.POLICIES[policy]
    amp.amp_index_set_tuning(mid["h"], [])
    ref = amp.amp_search(mid["h"], mid["Q"], 10, 16, policy=policy, bits=bits)
    for sch in SCHEDULES:
        amp.amp_index_set_tuning(mid["h"], [dict(sch, policy_kind=kind, nq_log2=7)])
        got = amp.amp_search(mid["h"], mid["Q"], 10, 16, policy=policy, bits=bits)
        assert np.array_equal(got["ids"], ref["ids"]), sch
        assert np.array_equal(got["dist"].view(np.uint32), ref["dist"].view(np.uint32)), sch
        if policy != "fp32":
            assert np.array_equal(got["qdist"], ref["qdist"]), sch
    amp.amp_index_set_tuning(mid["h"], [])


def test_autotune_records_the_fastest_schedule(mid):
    amp.amp_index_set_tuning(mid["h"], [])
    ref = amp.amp_search(mid["h"], mid["Q"], 10, 16, policy="fixed", bits=8)
    e = amp.amp_index_autotune(mid["h"], mid["Q"], 10, 16, policy="fixed", bits=8, repeats=3)
    assert e["policy_kind"] == amp.AMP_POLICY_FIXED and e["nq_log2"] == 7
    assert e["trials"] >= 7 and 0 < e["ms"] <= e["ms_default"]
    assert amp.amp_index_get_tuning(mid["h"]) == [e]
    got = amp.amp_search(mid["h"], mid["Q"], 10, 16, policy="fixed", bits=8)
    assert np.array_equal(got["ids"], ref["ids"]) and np.array_equal(got["qdist"], ref["qdist"])
    # a second call for the same bucket replaces the entry; another bucket adds one
    amp.amp_index_autotune(mid["h"], mid["Q"][:40], 10, 16, policy="fixed", bits=8, repeats=1)
    tab = amp.amp_index_get_tuning(mid["h"])
    assert sorted(x["nq_log2"] for x in tab) == [6, 7]
    amp.amp_index_set_tuning(mid["h"], [])
