"""The 256 GiB segregated-fit heap (one wavefront, 50 M requests) on the GPU,
on the lean core and on the ordered core.

Its tables peak at about 2,100 free and 13,300 live blocks, so the call asks
for capacities of 4,096 / 16,384.  The lean core keeps both tables in one
wave's LDS (1,920 free entries past the four register chunks, 16,384 live
entries); the ordered core keeps its chunks, records and the first 10,624
live entries in a 158 KiB pool and the rest in device memory.

The prefix test compares every result and the final state with the oracle.
The full-length test compares digests of all 50 M results and of the final
state, and sampled results, with tests/golden/large_seg_fit_256GiB.json,
written from the oracle by tests/golden/make_golden.py.
"""
import hashlib
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import oracle  # noqa: E402
from paper_2405_07079_amd import hda  # noqa: E402
from paper_2405_07079_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING = hda.tuning(heaps_per_group=1, reg_free=4, lds_free=1920, lds_live=16384)
META_FREE, META_LIVE = 4096, 16384


def say(*a):
    print(*a, flush=True)


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, "<i8").tobytes()).hexdigest()


def prefix(b, n):
    return W.Batch(b.name, b.arena, b.align, b.algo, np.array([0, n], np.int64),
                   np.ascontiguousarray(b.req[:n]), dict(b.meta))


# the ordered core: one wave owning a workgroup's LDS (158 KiB)
ORDERED = hda.tuning(heavy_heaps=1, heavy_kib=158)


def run(batch, tuning=TUNING):
    db = hda.upload(batch, tuning=tuning, meta_free=META_FREE, meta_live=META_LIVE)
    r = hda.hda_replay_resolve(db)
    assert r["lds_live"] == 16384 if tuning is TUNING else r["heavy_heaps"] == 1
    hda.hda_replay(db)
    torch.cuda.synchronize()
    return db.res.cpu().numpy(), hda.states_to_host(db)[0], int(db.status[0].item())


@pytest.fixture(scope="module")
def large():
    return W.large_seg_fit()


@pytest.mark.parametrize("core", ("lean", "ordered"))
def test_large_seg_fit_prefix(large, core):
    n = 2_000_000
    b = prefix(large, n)
    say(f"case: 256 GiB segregated fit, first {n} requests, {core} core")
    res, st, status = run(b, TUNING if core == "lean" else ORDERED)
    ores, ost = oracle.replay_heap(W.SEG_FIT, int(b.arena[0]), int(b.align[0]), b.req)
    assert status == 0
    if not np.array_equal(res, ores):
        i = int(np.nonzero(res != ores)[0][0])
        raise AssertionError(f"request {i}: gpu {res[i]} oracle {ores[i]}")
    assert np.array_equal(st, ost)


@pytest.mark.parametrize("core", ("lean", "ordered"))
def test_large_seg_fit_full_length(large, core):
    with open(os.path.join(HERE, "golden", "large_seg_fit_256GiB.json")) as f:
        g = json.load(f)
    assert digest(large.req) == g["trace_sha256"]
    say(f"case: 256 GiB segregated fit, 50 M requests, {core} core")
    res, st, status = run(large, TUNING if core == "lean" else ORDERED)
    assert status == 0
    pos = np.array(g["sample_positions"])
    assert np.array_equal(res[pos], np.array(g["sample_results"]))
    parsed = oracle.parse_state(st, W.SEG_FIT)
    assert len(parsed["free"]) == g["final_free_blocks"]
    assert len(parsed["live"]) == g["final_live_blocks"]
    assert digest(res) == g["results_sha256"]
    assert digest(st) == g["state_sha256"]
