"""The ordered core (free blocks in address-ordered chunks with a directory in
VGPRs) on the GPU, in its own launch beside the other heaps', against the
CPU oracle element by element (integers: exact) and against the other
cores' results.

Every test calls the library through its C ABI (the ctypes binding)."""
import numpy as np
import pytest

import oracle
from paper_2405_07079_amd import hda
from paper_2405_07079_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ALGOS = (0, 1, 2, 3, 4)


def say(*a):
    print(*a, flush=True)


def heavy(n, kib=0, **kw):
    return hda.tuning(heavy_heaps=n, heavy_kib=kib, **kw)


def gpu_replay(batch, tuning, meta_free=4096, meta_live=8192, order="lpt"):
    db = hda.upload(batch, order=order, tuning=tuning, meta_free=meta_free,
                    meta_live=meta_live)
    hda.hda_replay(db)
    torch.cuda.synchronize()
    return db.res.cpu().numpy()[:batch.requests], hda.states_to_host(db), db.status.cpu().numpy()


def check_against_oracle(batch, res, states, status):
    ores, ostates, _ = oracle.replay_batch(batch, threads=8)
    for h in range(batch.heaps):
        a, b = batch.req_off[h], batch.req_off[h + 1]
        if not np.array_equal(res[a:b], ores[a:b]):
            bad = int(np.nonzero(res[a:b] != ores[a:b])[0][0])
            raise AssertionError(f"heap {h} (algo {batch.algo[h]}) request {bad}: "
                                 f"gpu {res[a + bad]} oracle {ores[a + bad]}")
        assert status[h] == 0, (h, status[h])
        assert np.array_equal(states[h], ostates[h]), f"heap {h} state differs"


def tiny_blocks(algo, n, seed=7):
    """One heap of many small blocks in a 16 MiB arena at 16 B: thousands of
    free blocks that never merge away, so the chunks split, merge and share
    entries and the directory outgrows its first register (next fit passes
    2,048 free blocks by the end)."""
    return W.uniform_batch(seed=seed, heaps=1, arena=1 << 24, align=16, n=n, p_alloc=0.56,
                           lo=16, hi=160, algo=algo, name="tiny_blocks")


@pytest.mark.parametrize("algo", ALGOS)
def test_every_heap_on_the_ordered_core(algo):
    b = W.uniform_batch(seed=2, heaps=40, n=20_000, algo=algo)
    say(f"case: ordered core, 40 x 16 MiB heaps, 20k requests, algo {algo}, all heavy")
    res, states, status = gpu_replay(b, heavy(40))
    check_against_oracle(b, res, states, status)


@pytest.mark.parametrize("kib", (16, 158))
def test_mixed_batch_split_between_launches(kib):
    """The longest heaps of a mixed batch on the ordered core, the rest on the
    lean core in the launch beside it; with a 16 KiB pool most chunks and
    live entries of the ordered heaps are in device memory."""
    parts = [W.uniform_batch(seed=5 + a, heaps=6, n=int(3000 + 4000 * a), algo=a)
             for a in ALGOS]
    parts += [tiny_blocks(a, 12_000, seed=20 + a) for a in ALGOS]
    b = W.concat(parts, "mixed")
    say(f"case: mixed batch {b.heaps} heaps, 12 heaviest on the ordered core, pool {kib} KiB")
    res, states, status = gpu_replay(b, heavy(12, kib))
    check_against_oracle(b, res, states, status)


@pytest.mark.parametrize("algo", ALGOS)
def test_thousands_of_free_blocks(algo):
    b = tiny_blocks(algo, 60_000)
    say(f"case: ordered core, tiny blocks, 60k requests, algo {algo}")
    res, states, status = gpu_replay(b, heavy(1, 158), meta_live=65536)
    check_against_oracle(b, res, states, status)
    if algo == W.NEXT_FIT:
        assert oracle.parse_state(states[0], algo)["free"].__len__() > 2048


def test_capacity_exhausted_like_the_lean_core():
    """meta_free / meta_live reached: HDA_E_NOMETA at the same requests and
    the same final states as on the lean core."""
    b = W.concat([W.uniform_batch(seed=9, heaps=4, n=6000, algo=a) for a in ALGOS], "cap")
    want = gpu_replay(b, hda.tuning(), meta_free=64, meta_live=192)
    got = gpu_replay(b, heavy(b.heaps, 32), meta_free=64, meta_live=192)
    say("case: ordered core at capacity, statuses", sorted(set(got[2].tolist())))
    assert (want[2] == hda.HDA_E_NOMETA).any()
    assert np.array_equal(got[0], want[0])
    assert np.array_equal(got[2], want[2])
    for h in range(b.heaps):
        assert np.array_equal(got[1][h], want[1][h]), f"heap {h} state differs"


def test_max_arena_edges_on_the_ordered_core():
    b = W.max_arena_batch()
    say(f"case: 2^32 - 1 granule arenas on the ordered core, {b.heaps} heaps")
    res, states, status = gpu_replay(b, heavy(b.heaps, 32))
    check_against_oracle(b, res, states, status)


def test_uneven_batch_reduced_with_heavy_heaps():
    b = W.uneven_batch(heaps=512, len_scale=0.1)
    say(f"case: uneven batch, {b.heaps} heaps, {b.requests} requests, 32 on the ordered core")
    res, states, status = gpu_replay(b, heavy(32))
    check_against_oracle(b, res, states, status)


def test_graph_with_heavy_heaps_matches_eager():
    parts = [W.uniform_batch(seed=3 + a, heaps=8, n=5000, algo=a) for a in ALGOS]
    b = W.concat(parts, "graph")
    db = hda.upload(b, tuning=heavy(10, 32))
    hda.hda_replay(db)
    torch.cuda.synchronize()
    want = db.res.cpu().numpy().copy(), [s.copy() for s in hda.states_to_host(db)]
    g = hda.ReplayGraph(db)
    try:
        for k in range(3):
            say(f"case: graph with heavy heaps, replay {k}")
            db.res.fill_(0x5a5a)
            db.state.fill_(-5)
            g.launch()
            torch.cuda.synchronize()
            assert np.array_equal(db.res.cpu().numpy(), want[0])
            got = hda.states_to_host(db)
            for h in range(b.heaps):
                assert np.array_equal(got[h], want[1][h])
    finally:
        g.close()


def test_heavy_tuning_is_validated():
    b = W.uniform_batch(seed=2, heaps=4, n=100)
    for tu, mf in ((heavy(-1), 4096), (heavy(2, 8), 4096), (heavy(2, 4096), 4096),
                   (heavy(2), 8192)):
        db = hda.upload(b, tuning=(0,) * 6, meta_free=mf)
        db.tuning = tu
        with pytest.raises(hda.HdaError):
            hda.hda_replay(db)
    db = hda.upload(b, tuning=heavy(2))
    with pytest.raises(hda.HdaError) as e:
        hda.hda_replay_static(db)
    assert e.value.code == hda.HDA_E_INVAL
