"""GPU batched replay vs the CPU oracle, element by element (integers: exact).

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


def gpu_replay(batch, tuning=(0, 0, 0, 0, 0, 0), meta_free=4096, meta_live=8192,
               per_heap=False, order="lpt", with_state=True):
    db = hda.upload(batch, order=order, tuning=tuning, meta_free=meta_free,
                    meta_live=meta_live, with_state=with_state)
    (hda.hda_replay_per_heap if per_heap else hda.hda_replay)(db)
    torch.cuda.synchronize()
    states = hda.states_to_host(db) if with_state else None
    return db.res.cpu().numpy()[:batch.requests], states, db.status.cpu().numpy()


def check_against_oracle(batch, res, states, status, heaps=None):
    heaps = list(range(batch.heaps)) if heaps is None else list(heaps)
    sub = batch.subset(heaps)
    ores, ostates, _ = oracle.replay_batch(sub, threads=8)
    for k, h in enumerate(heaps):
        a, b = batch.req_off[h], batch.req_off[h + 1]
        got = res[a:b]
        exp = ores[sub.req_off[k]:sub.req_off[k + 1]]
        if not np.array_equal(got, exp):
            bad = int(np.nonzero(got != exp)[0][0])
            raise AssertionError(f"heap {h} (algo {batch.algo[h]}) request {bad}: "
                                 f"gpu {got[bad]} oracle {exp[bad]} req {batch.req[a + bad]}")
        assert status[h] == 0, (h, status[h])
        if states is not None:
            assert np.array_equal(states[h], ostates[k]), f"heap {h} state differs"


def test_single_heap_64KiB_all_algorithms():
    base = W.single_heap()
    b = W.concat([base.with_algo(a) for a in ALGOS], "single_heap x4")
    say("case: single heap 64 KiB, 10k requests, algos", ALGOS)
    res, states, status = gpu_replay(b)
    check_against_oracle(b, res, states, status)


def random_small_batch(seed, heaps, max_len=1500):
    rng = np.random.default_rng(seed)
    parts = []
    for h in range(heaps):
        gran = int(rng.integers(1, 300))
        align = int(1 << rng.integers(0, 13))
        n = int(rng.integers(0, max_len)) if h % 17 else 0
        algo = int(rng.integers(0, 5))
        parts.append(W.random_tiny(int(rng.integers(1 << 30)), n, gran, align=align,
                                   p_alloc=float(rng.uniform(0.4, 0.75)), algo=algo,
                                   max_granules=max(1, gran // int(rng.integers(1, 8)))))
    return W.concat(parts, "random_small")


def test_random_small_heaps_mixed():
    b = random_small_batch(11, 600)
    say("case: 600 random small heaps, mixed algorithms/alignments, some empty")
    res, states, status = gpu_replay(b)
    check_against_oracle(b, res, states, status)


def c2_like(heaps, n, algo):
    return W.uniform_batch(seed=2, heaps=heaps, n=n, algo=algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_16MiB_heaps_reduced(algo):
    b = c2_like(48, 30_000, algo)
    say(f"case: 48 x 16 MiB heaps, 30k requests, algo {algo}, default tuning")
    res, states, status = gpu_replay(b)
    check_against_oracle(b, res, states, status)


SPILL_TUNINGS = {
    # general core: LDS, then device memory
    "general_lds64": hda.tuning(heaps_per_group=2, reg_free=-1, reg_live=-1, lds_free=64,
                                lds_live=64),
    "general_no_lds": hda.tuning(heaps_per_group=4, reg_free=-1, reg_live=-1, lds_free=-1,
                                 lds_live=-1),
    # lean core with tiers too small for these heaps: every heap outgrows
    # them and moves to the general core mid-trace
    "lean_overflow": hda.tuning(heaps_per_group=2, reg_free=4, lds_free=-1, lds_live=64),
    "lean_lds_overflow": hda.tuning(heaps_per_group=4, reg_free=4, reg_live=-1, lds_free=64,
                                    lds_live=128),
}


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("where", sorted(SPILL_TUNINGS))
def test_spill_to_device_memory(algo, where):
    """Small register and LDS parts: most of each table spills to device
    memory, and entries move between registers, LDS and device memory."""
    b = c2_like(24, 20_000, algo)
    say(f"case: 24 x 16 MiB heaps, 20k requests, algo {algo}, tables {where}")
    res, states, status = gpu_replay(b, tuning=SPILL_TUNINGS[where])
    check_against_oracle(b, res, states, status)


@pytest.mark.parametrize("where", ("default", "general_no_lds"))
def test_max_arena_edges(where):
    """Arenas of 2^32 - 1 granules (a block ending at granule ~0, a free
    block of size 2^32 - 1) on the lean and the general core."""
    b = W.max_arena_batch()
    say(f"case: 2^32 - 1 granule arenas, {b.heaps} heaps, tables {where}")
    tu = hda.tuning() if where == "default" else SPILL_TUNINGS[where]
    res, states, status = gpu_replay(b, tuning=tu, meta_free=64, meta_live=64)
    check_against_oracle(b, res, states, status)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("where", ("default", "lean_overflow", "general_lds64"))
def test_partial_frees(algo, where):
    """Half the frees are partial (the victim keeps a head; segregated fit
    ignores the cut), on the lean core, through the move to the general core,
    and on the general core alone."""
    b = W.uniform_batch(seed=6, heaps=24, n=20_000, algo=algo, p_partial=0.5)
    say(f"case: 24 x 16 MiB heaps, 20k requests, half the frees partial, algo {algo}, "
        f"tables {where}")
    tu = hda.tuning() if where == "default" else SPILL_TUNINGS[where]
    res, states, status = gpu_replay(b, tuning=tu)
    check_against_oracle(b, res, states, status)


def test_tuning_does_not_change_results():
    b = W.concat([c2_like(16, 8000, a) for a in ALGOS], "mixed")
    ref = None
    for tu in (hda.tuning(), hda.tuning(heaps_per_group=1, reg_free=-1, reg_live=-1),
               hda.tuning(heaps_per_group=8, reg_free=-1, lds_free=128, lds_live=256),
               hda.tuning(heaps_per_group=16, lds_free=64, lds_live=512, groups=3),
               hda.tuning(heaps_per_group=2, reg_free=4, lds_free=-1, lds_live=64,
                          groups=1),
               hda.tuning(heaps_per_group=4, reg_free=4, reg_live=-1, lds_live=2048)):
        say("case: tuning", tu)
        res, states, status = gpu_replay(b, tuning=tu)
        assert (status == 0).all()
        if ref is None:
            ref = (res, states)
            check_against_oracle(b, res, states, status)
        else:
            assert np.array_equal(res, ref[0])
            assert all(np.array_equal(x, y) for x, y in zip(states, ref[1]))


@pytest.mark.parametrize("where", ("default", "lean_overflow"))
def test_per_heap_launch_matches_batched(where):
    b = W.concat([c2_like(6, 5000, a) for a in ALGOS], "mixed")
    tu = hda.tuning() if where == "default" else SPILL_TUNINGS[where]
    say(f"case: per-heap launches, 24 heaps, tuning {where}")
    r1, s1, st1 = gpu_replay(b, tuning=tu)
    r2, s2, st2 = gpu_replay(b, tuning=tu, per_heap=True)
    assert np.array_equal(r1, r2)
    assert all(np.array_equal(x, y) for x, y in zip(s1, s2))
    check_against_oracle(b, r2, s2, st2)


def test_uneven_batch_reduced():
    b = W.uneven_batch(heaps=2048, len_scale=0.02)
    say(f"case: uneven batch 2048 heaps, {b.requests} requests")
    res, states, status = gpu_replay(b)
    rng = np.random.default_rng(0)
    lens = np.diff(b.req_off)
    heaps = sorted(set(rng.choice(b.heaps, 200, replace=False).tolist())
                   | set(np.argsort(-lens)[:8].tolist()))
    check_against_oracle(b, res, states, status, heaps)


@pytest.mark.parametrize("bad", (dict(reg_free=3), dict(reg_free=8), dict(reg_live=4),
                                 dict(lds_free=100),
                                 dict(heaps_per_group=17), dict(lds_live=1 << 20)))
def test_bad_tuning_is_rejected(bad):
    db = hda.upload(c2_like(2, 100, 0), tuning=(0,) * 6)
    db.tuning = hda.tuning(**bad)
    with pytest.raises(hda.HdaError) as e:
        hda.hda_replay_resolve(db)
    assert e.value.code == hda.HDA_E_INVAL


def test_bad_heap_parameters():
    good = W.random_tiny(1, 50, 32, align=16)
    bad = []
    for A, g, algo in ((1000, 16, 0), (1024, 24, 0), (1024, 16, 7), (0, 16, 1),
                       (1 << 40, 16, 2)):
        b = W.random_tiny(2, 40, 8, align=16)
        b.arena[:] = A
        b.align[:] = g
        b.algo[:] = algo
        bad.append(b)
    batch = W.concat([good] + bad + [good], "bad")
    say("case: heaps with invalid parameters")
    res, states, status = gpu_replay(batch)
    assert status.tolist() == [0, -2, -2, -2, -2, -2, 0]
    for h in range(1, 6):
        a, b_ = batch.req_off[h], batch.req_off[h + 1]
        assert (res[a:b_] == hda.HDA_E_INVAL).all()
    check_against_oracle(batch, res, states, status, [0, 6])


def test_state_slot_too_small():
    b = c2_like(2, 3000, 3)
    db = hda.upload(b)
    so = db.state_off.cpu().numpy()
    so[1] = so[0] + 10          # heap 0 gets a 10-word slot
    db.state_off = torch.from_numpy(so).cuda()
    say("case: state slot too small")
    hda.hda_replay(db)
    torch.cuda.synchronize()
    st = db.status.cpu().numpy()
    assert st[0] == hda.HDA_E_RANGE and st[1] == 0
    need = int(db.state_len[0].item())
    _, ostates, _ = oracle.replay_batch(b.subset([0]))
    assert need == len(ostates[0])


def test_metadata_capacity_exhausted():
    """A heap whose live set outgrows its table gets HDA_E_NOMETA for the
    requests that would need a new entry; earlier results are unaffected."""
    b = c2_like(2, 4000, 2)
    say("case: live-table capacity 64")
    res, states, status = gpu_replay(b, tuning=hda.tuning(heaps_per_group=1), meta_free=64,
                                     meta_live=64)
    ores, _, _ = oracle.replay_batch(b, want_state=False)
    assert (status == hda.HDA_E_NOMETA).all()
    for h in range(2):
        a, e = b.req_off[h], b.req_off[h + 1]
        first = int(np.nonzero(res[a:e] == hda.HDA_E_NOMETA)[0][0])
        assert np.array_equal(res[a:a + first], ores[a:a + first])
        # the live table never exceeds its capacity
        st = oracle.parse_state(states[h], 2)
        assert len(st["live"]) <= 64 and len(st["free"]) <= 64


def test_empty_batch_and_empty_heaps():
    b = W.random_tiny(3, 0, 16)
    say("case: empty traces")
    res, states, status = gpu_replay(W.concat([b, b, b]))
    assert res.size == 0 and (status == 0).all()
    st = oracle.parse_state(states[0], 0)
    assert st["free"] == [(0, 256)] and st["live"] == []
    db = hda.upload(W.concat([b]))
    db.n_heaps = 0
    hda.hda_replay(db)
    torch.cuda.synchronize()


def test_graph_replays_match_eager():
    """A captured replay, launched several times with eager work between the
    launches, rewrites every output each time exactly as the eager call."""
    b = W.concat([c2_like(8, 6000, a) for a in ALGOS], "mixed")
    say("case: hipGraph of one replay call, 3 launches")
    ref_res, ref_states, ref_status = gpu_replay(b)
    db = hda.upload(b)
    g = hda.ReplayGraph(db)
    other = hda.upload(c2_like(4, 3000, 3))
    try:
        for k in range(3):
            db.res.fill_(0x5a5a)
            db.status.fill_(77)
            db.state.fill_(-9)
            g.launch()
            torch.cuda.synchronize()
            assert np.array_equal(db.res.cpu().numpy()[:b.requests], ref_res), f"launch {k}"
            assert np.array_equal(db.status.cpu().numpy(), ref_status)
            got = hda.states_to_host(db)
            assert all(np.array_equal(x, y) for x, y in zip(got, ref_states))
            hda.hda_replay(other)            # eager work between launches
            torch.cuda.synchronize()
    finally:
        g.close()


def test_autotune_picks_a_valid_tuning():
    b = W.uneven_batch(heaps=512, len_scale=0.01)
    say(f"case: autotune on an uneven batch, {b.requests} requests")
    db = hda.upload(b)
    db.res.fill_(0x5a5a)
    tu = hda.hda_replay_autotune(db)
    assert tu[1] > 0 and tu[3] > 0 and tu[4] > 0        # lean path, LDS pool
    assert (db.res == 0x5a5a).all()                     # the caller's buffers are untouched
    hda.retune(db, tu)
    hda.hda_replay(db)
    torch.cuda.synchronize()
    res = db.res.cpu().numpy()[:b.requests]
    rng = np.random.default_rng(1)
    lens = np.diff(b.req_off)
    heaps = sorted(set(rng.choice(b.heaps, 60, replace=False).tolist())
                   | set(np.argsort(-lens)[:6].tolist()))
    check_against_oracle(b, res, hda.states_to_host(db), db.status.cpu().numpy(), heaps)


def test_autotune_reuses_its_choice_for_the_same_shape():
    """A second call on a batch of the same shape (here: the same batch,
    and a copy with other requests but the same lengths and heaps) returns
    the first call's choice from the cache, without timing again."""
    import time
    b = W.uneven_batch(heaps=384, len_scale=0.01, seed=13)
    say(f"case: autotune cache, {b.heaps} heaps")
    db = hda.upload(b)
    t0 = time.perf_counter()
    first = hda.hda_replay_autotune(db)
    t1 = time.perf_counter()
    again = hda.hda_replay_autotune(db)
    t2 = time.perf_counter()
    assert again == first
    assert t2 - t1 < 0.5 * (t1 - t0)
    other = W.Batch(b.name, b.arena, b.align, b.algo, b.req_off,
                    np.where(b.req >= 0, b.req // 2 + 1, b.req), dict(b.meta))
    assert hda.hda_replay_autotune(hda.upload(other)) == first
