"""The bitmask allocator (one flag per granule, next-fit scan; Sec. III-B)
on the GPU through hda_bitmap_replay, against the oracle element by element
(results and final states)."""
import numpy as np
import pytest

import oracle
from paper_2405_07079_amd import hda
from paper_2405_07079_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BM = 5


def say(*a):
    print(*a, flush=True)


def run(batch, max_gran=None, meta_live=8192):
    db = hda.upload(batch, meta_live=meta_live)
    hda.hda_bitmap_replay(db, max_gran or hda.max_granules(batch))
    torch.cuda.synchronize()
    return (db.res.cpu().numpy()[:batch.requests], hda.states_to_host(db),
            db.status.cpu().numpy())


def check(batch, res, states, status):
    ores, ostates, _ = oracle.replay_batch(batch, threads=8)
    for h in range(batch.heaps):
        a, b = batch.req_off[h], batch.req_off[h + 1]
        if not np.array_equal(res[a:b], ores[a:b]):
            i = int(np.nonzero(res[a:b] != ores[a:b])[0][0])
            raise AssertionError(f"heap {h} request {i}: gpu {res[a + i]} oracle {ores[a + i]}")
        assert status[h] == 0, (h, status[h])
        assert np.array_equal(states[h], ostates[h]), f"heap {h} state"


def test_random_small_heaps():
    rng = np.random.default_rng(31)
    parts = []
    for h in range(300):
        gran = int(rng.integers(1, 3000))
        n = int(rng.integers(0, 800)) if h % 13 else 0
        parts.append(W.random_tiny(int(rng.integers(1 << 30)), n, gran,
                                   align=int(1 << rng.integers(0, 10)), algo=BM,
                                   max_granules=max(1, gran // int(rng.integers(1, 8))),
                                   p_partial=float(rng.uniform(0, 0.5))))
    b = W.concat(parts)
    say(f"case: {b.heaps} small bitmask heaps, {b.requests} requests")
    check(b, *run(b))


def test_16MiB_heaps_reduced():
    b = W.uniform_batch(seed=7, heaps=48, n=10_000, algo=BM, p_partial=0.1)
    say(f"case: 48 x 16 MiB bitmask heaps (262,144 granules), 10k requests")
    check(b, *run(b))


def test_more_than_64_nodes():
    """Arenas past 262,144 granules: the node summaries take several steps
    of 64, and runs span nodes."""
    parts = [W.random_tiny(40 + k, 3000, g, align=16, algo=BM, max_granules=hi,
                           p_partial=0.1)
             for k, (g, hi) in enumerate(((300_000, 4), (600_000, 60_000),
                                          (1_500_000, 200_000), (262_145, 5000)))]
    b = W.concat(parts)
    say(f"case: {b.heaps} bitmask heaps of 262,145-1,500,000 granules, {b.requests} requests")
    check(b, *run(b))


def test_max_arena():
    """The largest arena, 2^32 - 1 granules of 64 B (256 GiB of flags' worth,
    512 MiB of flags): ragged last word and node, blocks that end at the
    arena's last granule, whole-arena requests, wrapping searches (the two
    hand-written traces the table kernels are tested on at this size)."""
    mb = W.max_arena_batch()
    per_trace = mb.heaps // 2
    b = mb.subset([0, per_trace]).with_algo(BM)
    assert int(b.arena[0] // b.align[0]) == (1 << 32) - 1
    say(f"case: 2 bitmask heaps of 2^32 - 1 granules, {b.requests} requests")
    check(b, *run(b, meta_live=64))


def test_rejections_and_capacity():
    good = W.random_tiny(1, 200, 500, align=16, algo=BM)
    other = W.random_tiny(2, 200, 500, align=16, algo=0)     # not a bitmask heap
    big = W.random_tiny(3, 50, 5000, align=16, algo=BM)       # over max_granules
    b = W.concat([good, other, big])
    say("case: rejected heaps")
    res, states, status = run(b, max_gran=1000)
    assert status.tolist() == [0, -2, -2]
    assert (res[b.req_off[1]:] == -2).all()
    check(W.concat([good]), res[:b.req_off[1]], states[:1], status[:1])
    # the table kernels reject bitmask heaps
    db = hda.upload(W.concat([good]))
    hda.hda_replay(db)
    torch.cuda.synchronize()
    assert int(db.status[0].item()) == -2
    # live table capacity
    cap = W.random_tiny(4, 400, 256, align=16, p_alloc=0.85, algo=BM, max_granules=4)
    res, _, status = run(cap, meta_live=64)
    assert status[0] == -4
    ores, _ = oracle.replay_heap(BM, int(cap.arena[0]), int(cap.align[0]), cap.req)
    k = int(np.nonzero(res == -4)[0][0])
    assert np.array_equal(res[:k], ores[:k])
