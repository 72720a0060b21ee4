"""Full-size workloads on the GPU, in the launch configuration the benchmark
uses, compared with the oracle on EVERY heap: every result and every final
state, element by element (the oracle replays the whole batch on all host
threads).

* 4,096 heaps x 100,000 requests (16 MiB arenas), best fit, segregated
  fit and TLSF, default tuning, states dumped.
* The same batch on best fit with 2 % of the frees partial, and replayed by
  the bitmask allocator.
* The uneven batch (16,384 heaps, 46.9 M requests), autotuned and launched
  as a captured graph.

The service at full load is in test_gpu_zservice_full_load.py.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2405_07079_amd import hda
from paper_2405_07079_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def host_threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 8


def check_every_heap(batch, db, state_blocks):
    """Results, statuses and states of all heaps against the oracle."""
    res = db.res[:batch.requests].cpu().numpy()
    status = db.status.cpu().numpy()
    so = db.state_off.cpu().numpy()
    sl = db.state_len.cpu().numpy()
    state = db.state.cpu().numpy()
    say(f"  oracle: {batch.heaps} heaps, {batch.requests} requests, "
        f"{host_threads()} threads")
    ores, ostates, _ = oracle.replay_batch(batch, threads=host_threads(),
                                           state_blocks=state_blocks)
    bad = np.nonzero(status != 0)[0]
    assert bad.size == 0, f"heap {bad[0]} status {status[bad[0]]}"
    if not np.array_equal(res, ores):
        i = int(np.nonzero(res != ores)[0][0])
        h = int(np.searchsorted(batch.req_off, i, side="right") - 1)
        raise AssertionError(f"heap {h} (algo {batch.algo[h]}) request "
                             f"{i - batch.req_off[h]}: gpu {res[i]} oracle {ores[i]}")
    for h in range(batch.heaps):
        got = state[so[h]:so[h] + min(sl[h], so[h + 1] - so[h])]
        assert np.array_equal(got, ostates[h]), f"heap {h} (algo {batch.algo[h]}) state"
    say(f"  {batch.heaps} heaps equal the oracle")


META_FREE, META_LIVE = 4096, 8192


@pytest.fixture(scope="module")
def batch_4096():
    return W.uniform_batch()


@pytest.mark.parametrize("algo", (W.BEST_FIT, W.SEG_FIT, W.TLSF))
def test_4096_heaps_full_size(batch_4096, algo):
    b = batch_4096.with_algo(algo)
    say(f"case: 4096 x 16 MiB heaps, 100k requests each, algo {algo}")
    db = hda.upload(b, meta_free=META_FREE, meta_live=META_LIVE)
    hda.hda_replay(db)
    torch.cuda.synchronize()
    check_every_heap(b, db, META_FREE + META_LIVE)


def test_4096_heaps_bitmap_full_size(batch_4096):
    """The benchmark's bitmask-allocator leg: the same batch, one flag per
    granule."""
    b = batch_4096.with_algo(W.BITMAP)
    say("case: 4096 x 16 MiB heaps, 100k requests each, bitmask allocator")
    db = hda.upload(b, meta_live=META_LIVE)
    hda.hda_bitmap_replay(db, hda.max_granules(b))
    torch.cuda.synchronize()
    check_every_heap(b, db, 2 * META_LIVE + 1)


def test_4096_heaps_partial_frees_full_size():
    """The benchmark's partial-deallocation leg: best fit, 2 % of the frees
    partial, default tuning."""
    b = W.uniform_batch(algo=W.BEST_FIT, p_partial=0.02)
    say("case: 4096 x 16 MiB heaps, 100k requests each, best fit, 2 % partial frees")
    db = hda.upload(b, meta_free=META_FREE, meta_live=META_LIVE)
    hda.hda_replay(db)
    torch.cuda.synchronize()
    check_every_heap(b, db, META_FREE + META_LIVE)


def test_uneven_batch_full_size_autotuned_graph():
    b = W.uneven_batch()
    say(f"case: uneven batch, {b.heaps} heaps, {b.requests} requests, autotuned, graph")
    db = hda.upload(b, meta_free=META_FREE, meta_live=META_LIVE)
    hda.retune(db, hda.hda_replay_autotune(db))
    g = hda.ReplayGraph(db)
    try:
        db.res.fill_(0x5a5a)
        g.launch()
        torch.cuda.synchronize()
    finally:
        g.close()
    check_every_heap(b, db, META_FREE + META_LIVE)
