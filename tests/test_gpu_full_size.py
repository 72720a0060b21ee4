"""Full-size workloads on the GPU, in the launch configuration the benchmark
uses, checked on heaps the oracle replays one by one (and, for the service,
on properties that hold at any size).

* 4,096 heaps x 100,000 requests (16 MiB arenas), best fit, segregated
  fit and TLSF, default tuning, states dumped: 24 sampled heaps per algorithm
  (including the first and the last) compared element by element.
* The same batch on best fit with 2 % of the frees partial, and replayed by
  the bitmask allocator: 24 sampled heaps each.
* The uneven batch (16,384 heaps, 46.9 M requests), autotuned and launched
  as a captured graph: 48 sampled heaps plus the 4 longest.
* The service under 1e7 requests/s from 100,000 clients (one heap each):
  every request completes without error, throughput follows the offered
  rate, p50 latency is finite.
"""
import numpy as np
import pytest

import oracle
from paper_2405_07079_amd import hda
from paper_2405_07079_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def check_heaps(batch, res, db, status, heaps):
    states = dict(zip(heaps, hda.states_to_host(db, heaps)))
    sub = batch.subset(heaps)
    ores, ostates, _ = oracle.replay_batch(sub, threads=16)
    for k, h in enumerate(heaps):
        a, b = batch.req_off[h], batch.req_off[h + 1]
        got, exp = res[a:b], ores[sub.req_off[k]:sub.req_off[k + 1]]
        if not np.array_equal(got, exp):
            i = int(np.nonzero(got != exp)[0][0])
            raise AssertionError(f"heap {h} algo {batch.algo[h]} request {i}: "
                                 f"gpu {got[i]} oracle {exp[i]}")
        assert status[h] == 0, (h, status[h])
        assert np.array_equal(states[h], ostates[k]), f"heap {h} state"


@pytest.fixture(scope="module")
def batch_4096():
    return W.uniform_batch()


@pytest.mark.parametrize("algo", (W.BEST_FIT, W.SEG_FIT, W.TLSF))
def test_4096_heaps_full_size_sampled(batch_4096, algo):
    b = batch_4096.with_algo(algo)
    say(f"case: 4096 x 16 MiB heaps, 100k requests each, algo {algo}")
    db = hda.upload(b)
    hda.hda_replay(db)
    torch.cuda.synchronize()
    status = db.status.cpu().numpy()
    assert (status == 0).all()
    rng = np.random.default_rng(100 + algo)
    heaps = sorted(set(rng.choice(b.heaps, 22, replace=False).tolist()) | {0, b.heaps - 1})
    res = np.empty(b.requests, np.int64)
    for h in heaps:   # copy only the sampled heaps' results back
        a, e = int(b.req_off[h]), int(b.req_off[h + 1])
        res[a:e] = db.res[a:e].cpu().numpy()
    check_heaps(b, res, db, status, heaps)


def test_4096_heaps_bitmap_full_size_sampled(batch_4096):
    """The benchmark's bitmask-allocator leg: the same batch, one flag per
    granule; 24 sampled heaps element by element."""
    b = batch_4096.with_algo(W.BITMAP)
    say("case: 4096 x 16 MiB heaps, 100k requests each, bitmask allocator")
    db = hda.upload(b)
    hda.hda_bitmap_replay(db, hda.max_granules(b))
    torch.cuda.synchronize()
    status = db.status.cpu().numpy()
    assert (status == 0).all()
    rng = np.random.default_rng(55)
    heaps = sorted(set(rng.choice(b.heaps, 22, replace=False).tolist()) | {0, b.heaps - 1})
    res = np.empty(b.requests, np.int64)
    for h in heaps:
        a, e = int(b.req_off[h]), int(b.req_off[h + 1])
        res[a:e] = db.res[a:e].cpu().numpy()
    check_heaps(b, res, db, status, heaps)


def test_4096_heaps_partial_frees_full_size_sampled():
    """The benchmark's partial-deallocation leg: best fit, 2 % of the frees
    partial, default tuning; 24 sampled heaps element by element."""
    b = W.uniform_batch(algo=W.BEST_FIT, p_partial=0.02)
    say("case: 4096 x 16 MiB heaps, 100k requests each, best fit, 2 % partial frees")
    db = hda.upload(b)
    hda.hda_replay(db)
    torch.cuda.synchronize()
    status = db.status.cpu().numpy()
    assert (status == 0).all()
    rng = np.random.default_rng(77)
    heaps = sorted(set(rng.choice(b.heaps, 22, replace=False).tolist()) | {0, b.heaps - 1})
    res = np.empty(b.requests, np.int64)
    for h in heaps:
        a, e = int(b.req_off[h]), int(b.req_off[h + 1])
        res[a:e] = db.res[a:e].cpu().numpy()
    check_heaps(b, res, db, status, heaps)


def test_uneven_batch_full_size_autotuned_graph():
    b = W.uneven_batch()
    say(f"case: uneven batch, {b.heaps} heaps, {b.requests} requests, autotuned, graph")
    db = hda.upload(b)
    hda.retune(db, hda.hda_replay_autotune(db))
    g = hda.ReplayGraph(db)
    try:
        db.res.fill_(0x5a5a)
        g.launch()
        torch.cuda.synchronize()
    finally:
        g.close()
    status = db.status.cpu().numpy()
    assert (status == 0).all()
    res = db.res.cpu().numpy()[:b.requests]
    lens = np.diff(b.req_off)
    rng = np.random.default_rng(7)
    heaps = sorted(set(rng.choice(b.heaps, 48, replace=False).tolist())
                   | set(np.argsort(-lens)[:4].tolist()))
    check_heaps(b, res, db, status, heaps)


def test_service_at_full_load():
    say("case: service, 100,000 clients, 1e7 requests/s offered, 1 s measured")
    s = hda.Server(max_heaps=100_016, max_seconds=300)
    try:
        rep, _ = s.load(clients=100_000, rate=1e7, warmup_s=0.3, measure_s=1.0, threads=8)
    finally:
        s.stop()
    say("report", rep)
    assert rep["errors"] == 0
    assert rep["completed"] == rep["issued"] > 5_000_000
    assert rep["throughput"] > 0.9e7
    assert 0 < rep["p50_us"] <= rep["p99_us"] <= rep["max_us"]
    assert rep["alloc_ok"] > 0 and rep["frees"] > 0
