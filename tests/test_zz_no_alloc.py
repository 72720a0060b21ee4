"""hda_replay_static (the replay entry point that allocates nothing and runs
on the library's static per-GPU scratch) against hda_replay on the same
batch, through the C ABI: every result, status and final state identical
(integers, exact), and equal to the oracle.  Two calls in a row, the second
on a smaller batch, so the second runs on scratch the first left behind."""
import numpy as np
import pytest

import oracle
from paper_2405_07079_amd import hda
from paper_2405_07079_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def outputs(db, n):
    torch.cuda.synchronize()
    return (db.res.cpu().numpy()[:n].copy(), db.status.cpu().numpy().copy(),
            [s.copy() for s in hda.states_to_host(db)])


def poison(db):
    db.res.fill_(0x5a5a)
    db.status.fill_(77)
    db.state.fill_(-5)
    db.state_len.fill_(-1)


def run_both(batch, meta_free, meta_live):
    db = hda.upload(batch, meta_free=meta_free, meta_live=meta_live)
    assert hda.hda_replay_workspace(db) <= hda.STATIC_SCRATCH_BYTES
    hda.hda_replay(db)
    want = outputs(db, batch.requests)
    poison(db)
    hda.hda_replay_static(db)
    got = outputs(db, batch.requests)
    return want, got


def check(batch, want, got):
    assert np.array_equal(got[0], want[0]), "results differ from hda_replay"
    assert np.array_equal(got[1], want[1]), "statuses differ from hda_replay"
    for h in range(batch.heaps):
        assert np.array_equal(got[2][h], want[2][h]), f"heap {h} state differs"
    assert (got[1] == 0).all()
    ores, ostates, _ = oracle.replay_batch(batch, threads=8)
    assert np.array_equal(got[0], ores), "results differ from the oracle"
    for h in range(batch.heaps):
        assert np.array_equal(got[2][h], ostates[h]), f"heap {h} state differs from the oracle"


def test_static_scratch_matches_workspace_replay():
    big = W.concat([W.uniform_batch(heaps=48, n=4000, algo=a, seed=11 + a) for a in range(5)],
                   "no_alloc_big")
    small = W.concat([W.uniform_batch(heaps=6, n=1500, algo=a, seed=31 + a) for a in range(5)]
                     + [W.single_heap(n=2000).with_algo(a) for a in range(5)], "no_alloc_small")
    assert small.heaps < big.heaps and small.requests < big.requests
    say(f"case: static scratch, call 1: {big.heaps} heaps, {big.requests} requests")
    want, got = run_both(big, 4096, 8192)
    check(big, want, got)
    say(f"case: static scratch, call 2: {small.heaps} heaps, {small.requests} requests")
    want, got = run_both(small, 1024, 2048)
    check(small, want, got)


def test_static_scratch_rejects_oversized_plans():
    b = W.uniform_batch(heaps=4096, n=64)
    db = hda.upload(b, meta_free=4096, meta_live=8192)
    assert hda.hda_replay_workspace(db) > hda.STATIC_SCRATCH_BYTES
    say("case: static scratch, oversized plan (host-side rejection, nothing launched)")
    with pytest.raises(hda.HdaError) as e:
        hda.hda_replay_static(db)
    assert e.value.code == hda.HDA_E_RANGE
