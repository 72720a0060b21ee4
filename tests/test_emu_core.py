"""The device replay core, compiled for the CPU and run as a lockstep-emulated
wavefront (tests/emu), against the oracle.  This checks the kernel's own
logic (selection by wave reductions, swap-remove tables, push stamps, LDS /
spill split, capacity errors, state dump) without a GPU."""
import numpy as np
import pytest

import emu
import oracle
from paper_2405_07079_amd import workloads as W

ALGOS = (0, 1, 2, 3, 4)


def check(batch, res, states, status, heaps=None):
    heaps = list(range(batch.heaps)) if heaps is None else list(heaps)
    sub = batch.subset(heaps)
    ores, ostates, _ = oracle.replay_batch(sub)
    for k, h in enumerate(heaps):
        a, b = batch.req_off[h], batch.req_off[h + 1]
        got, exp = res[a:b], ores[sub.req_off[k]:sub.req_off[k + 1]]
        if not np.array_equal(got, exp):
            i = int(np.nonzero(got != exp)[0][0])
            raise AssertionError(f"heap {h} algo {batch.algo[h]} request {i}: "
                                 f"emulated {got[i]} oracle {exp[i]}")
        assert status[h] == 0
        assert np.array_equal(states[h], ostates[k]), f"heap {h} state"


@pytest.mark.parametrize("algo", ALGOS)
def test_single_heap_64KiB_register_tables(algo):
    b = W.single_heap(n=4000).with_algo(algo)
    res, states, status, _ = emu.replay(b, kf=64, kl=128, cf=4096, cl=8192, shape=2)
    check(b, res, states, status)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("shape", (0, 1))
def test_single_heap_spilling_tables(algo, shape):
    """Small register part and LDS part: entries cross registers, LDS and
    device memory."""
    b = W.single_heap(n=3000, seed=7).with_algo(algo)
    res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=4096, cl=4096, shape=shape)
    check(b, res, states, status)


def test_random_small_heaps():
    rng = np.random.default_rng(5)
    parts = []
    for h in range(40):
        gran = int(rng.integers(1, 120))
        parts.append(W.random_tiny(int(rng.integers(1 << 30)), int(rng.integers(0, 300)),
                                   gran, align=int(1 << rng.integers(0, 12)),
                                   algo=int(rng.integers(0, 5)),
                                   max_granules=max(1, gran // int(rng.integers(1, 6)))))
    b = W.concat(parts)
    res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=512, cl=512, shape=1)
    check(b, res, states, status)


@pytest.mark.parametrize("algo", ALGOS)
def test_16MiB_heap(algo):
    b = W.uniform_batch(heaps=1, n=2500, algo=algo)
    res, states, status, _ = emu.replay(b, kf=64, kl=128, cf=4096, cl=4096, shape=2)
    check(b, res, states, status)


def test_capacity_exhausted_changes_nothing():
    b = W.uniform_batch(heaps=1, n=1500, algo=2)
    res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=64, cl=64, shape=1)
    ores, _, _ = oracle.replay_batch(b, want_state=False)
    assert status[0] == -4
    first = int(np.nonzero(res == -4)[0][0])
    assert np.array_equal(res[:first], ores[:first])
    st = oracle.parse_state(states[0], 2)
    assert len(st["live"]) <= 64 and len(st["free"]) <= 64
    # a request refused for capacity leaves the state as it was: replaying the
    # accepted requests alone on the oracle gives the same final state
    acc = b.req[res != -4]
    h = oracle.Heap(2, int(b.arena[0]), int(b.align[0]))
    keep = h.replay(acc)
    assert np.array_equal(keep, res[res != -4])
    assert np.array_equal(h.state(), states[0])


def test_invalid_heap_parameters():
    good = W.random_tiny(1, 50, 32, align=16)
    bad = W.random_tiny(2, 40, 8, align=16)
    bad.arena[:] = 1000
    b = W.concat([good, bad, good])
    res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=256, cl=256)
    assert status.tolist() == [0, -2, 0]
    assert (res[b.req_off[1]:b.req_off[2]] == -2).all()
    check(b, res, states, status, heaps=[0, 2])


# ---- lean core (registers + LDS; a heap that outgrows them moves to the
# general core and continues there) ----

@pytest.mark.parametrize("algo", ALGOS)
def test_lean_single_heap_64KiB(algo):
    b = W.single_heap(n=4000).with_algo(algo)
    ovf = np.zeros(b.heaps, np.uint8)
    res, states, status, _ = emu.replay(b, kf=128, kl=1024, cf=4096, cl=8192, shape=4,
                                        overflowed=ovf)
    check(b, res, states, status)
    assert not ovf.any()


@pytest.mark.parametrize("algo", ALGOS)
def test_lean_16MiB_heap_cold_entries_in_lds(algo):
    """One register chunk: most free entries live in LDS."""
    b = W.uniform_batch(heaps=1, n=2500, algo=algo)
    ovf = np.zeros(b.heaps, np.uint8)
    res, states, status, _ = emu.replay(b, kf=512, kl=1024, cf=4096, cl=4096, shape=3,
                                        overflowed=ovf)
    check(b, res, states, status)
    assert not ovf.any()


@pytest.mark.parametrize("algo", ALGOS)
def test_lean_overflow_moves_to_general_core(algo):
    """Tiers far smaller than the tables: the heap's tables move into the
    general core's layout mid-trace and the replay continues there, with the
    same results."""
    b = W.uniform_batch(heaps=1, n=2000, algo=algo)
    ovf = np.zeros(b.heaps, np.uint8)
    res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=4096, cl=4096, shape=3,
                                        overflowed=ovf)
    check(b, res, states, status)
    assert ovf.all()


def test_lean_capacity_within_tiers_is_exact():
    """Capacities no larger than the tiers: E_NOMETA on the lean core itself,
    no move to the general core, results equal to the general core's."""
    b = W.uniform_batch(heaps=1, n=1500, algo=2)
    ovf = np.zeros(b.heaps, np.uint8)
    res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=64, cl=64, shape=3,
                                        overflowed=ovf)
    gres, gstates, gstatus, _ = emu.replay(b, kf=64, kl=64, cf=64, cl=64, shape=1)
    assert not ovf.any()
    assert status[0] == -4 == gstatus[0]
    assert np.array_equal(res, gres)
    assert np.array_equal(states[0], gstates[0])


def test_lean_random_small_heaps():
    rng = np.random.default_rng(11)
    parts = []
    for h in range(40):
        gran = int(rng.integers(1, 400))
        parts.append(W.random_tiny(int(rng.integers(1 << 30)), int(rng.integers(0, 400)),
                                   gran, align=int(1 << rng.integers(0, 12)),
                                   algo=int(rng.integers(0, 5)),
                                   max_granules=max(1, gran // int(rng.integers(1, 8)))))
    b = W.concat(parts)
    ovf = np.zeros(b.heaps, np.uint8)
    res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=512, cl=512, shape=3,
                                        overflowed=ovf)
    check(b, res, states, status)


def test_lean_invalid_heap_parameters():
    good = W.random_tiny(1, 50, 32, align=16)
    bad = W.random_tiny(2, 40, 8, align=16)
    bad.arena[:] = 1000
    b = W.concat([good, bad, good])
    res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=256, cl=256, shape=4)
    assert status.tolist() == [0, -2, 0]
    assert (res[b.req_off[1]:b.req_off[2]] == -2).all()
    check(b, res, states, status, heaps=[0, 2])


def test_max_arena_edges():
    """Arenas of 2^32 - 1 granules: a block can end at granule ~0 (the lean
    core's empty-slot address) and the whole free arena's size equals the
    32-bit "none" value.  General and lean cores, every algorithm."""
    b = W.max_arena_batch()
    for shape in (1, 3, 4):
        res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=64, cl=64, shape=shape)
        check(b, res, states, status)


# ---- partial deallocation (the sequential fits keep a head of the victim;
# segregated fit ignores the cut) ----

@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("shape", (1, 3, 4))
def test_partial_frees_16MiB_heap(algo, shape):
    b = W.uniform_batch(heaps=1, n=2500, algo=algo, p_partial=0.5)
    ovf = np.zeros(b.heaps, np.uint8)
    res, states, status, _ = emu.replay(b, kf=512, kl=1024, cf=4096, cl=4096, shape=shape,
                                        overflowed=ovf)
    check(b, res, states, status)
    assert not ovf.any()


@pytest.mark.parametrize("algo", ALGOS)
def test_partial_frees_lean_overflow(algo):
    """Tiers too small: the heap moves to the general core mid-trace with
    shrunk live entries in its tables."""
    b = W.uniform_batch(heaps=1, n=2000, algo=algo, p_partial=0.5)
    ovf = np.zeros(b.heaps, np.uint8)
    res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=4096, cl=4096, shape=3,
                                        overflowed=ovf)
    check(b, res, states, status)
    assert ovf.all()


def test_partial_frees_random_small_heaps():
    rng = np.random.default_rng(12)
    parts = []
    for h in range(40):
        gran = int(rng.integers(1, 400))
        parts.append(W.random_tiny(int(rng.integers(1 << 30)), int(rng.integers(0, 400)),
                                   gran, align=int(1 << rng.integers(0, 12)),
                                   algo=int(rng.integers(0, 5)),
                                   max_granules=max(1, gran // int(rng.integers(1, 8))),
                                   p_partial=float(rng.uniform(0.1, 1.0))))
    b = W.concat(parts)
    for shape in (1, 3):
        res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=512, cl=512, shape=shape)
        check(b, res, states, status)


# ---- the bitmask allocator (one flag per granule, next-fit scan) ----

def test_bitmap_random_small_heaps():
    rng = np.random.default_rng(21)
    parts = []
    for h in range(40):
        gran = int(rng.integers(1, 700))       # ragged word counts
        parts.append(W.random_tiny(int(rng.integers(1 << 30)), int(rng.integers(0, 300)),
                                   gran, align=int(1 << rng.integers(0, 8)), algo=5,
                                   max_granules=max(1, gran // int(rng.integers(1, 6))),
                                   p_partial=float(rng.uniform(0, 0.6))))
    b = W.concat(parts)
    res, states, status, _ = emu.replay(b, cf=1024, cl=1024, shape=5)
    check(b, res, states, status)


@pytest.mark.parametrize("granules,hi", ((5000, 200), (9000, 9000), (70_000, 3000),
                                         (600_000, 60_000), (300_000, 4)))
def test_bitmap_runs_across_words_and_steps(granules, hi):
    """Arenas of several 4,096-granule nodes, runs longer than a word or a
    node, and more than 64 nodes (node summaries read in several steps)."""
    b = W.random_tiny(granules, 600, granules, align=16, algo=5, max_granules=hi,
                      p_partial=0.2)
    res, states, status, _ = emu.replay(b, cf=4096, cl=4096, shape=5)
    check(b, res, states, status)


def test_bitmap_16MiB_heap():
    b = W.uniform_batch(heaps=1, n=1500, algo=5)
    res, states, status, _ = emu.replay(b, cf=4096, cl=4096, shape=5)
    check(b, res, states, status)


def test_bitmap_live_capacity():
    """A live table too small: E_NOMETA, results equal to the oracle's up to
    the first refusal."""
    b = W.random_tiny(3, 400, 256, align=16, p_alloc=0.8, algo=5, max_granules=4)
    res, states, status, _ = emu.replay(b, cf=4096, cl=16, shape=5)
    assert status[0] == -4
    ores, _ = oracle.replay_heap(5, int(b.arena[0]), int(b.align[0]), b.req)
    k = int(np.nonzero(res == -4)[0][0])
    assert np.array_equal(res[:k], ores[:k])


# ---- the ordered core (free blocks in address-ordered chunks, directory in
# VGPRs; shape 6: a pool of 8 KiB + kf * 16 + kl * 8 bytes, kf * 16 of them
# for chunk slots, the rest of each table in the device slot) ----

@pytest.mark.parametrize("algo", ALGOS)
def test_ordered_single_heap_64KiB(algo):
    b = W.single_heap(n=3000).with_algo(algo)
    res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=4096, cl=8192, shape=6)
    check(b, res, states, status)


@pytest.mark.parametrize("algo", ALGOS)
def test_ordered_many_free_blocks(algo):
    """Hundreds of free blocks of small sizes: chunks split at 64 entries,
    merge or share entries below 32, and most of them sit past the pool's
    slots in the device slot."""
    b = W.uniform_batch(seed=7, heaps=1, arena=1 << 24, align=16, n=9000, p_alloc=0.56,
                        lo=16, hi=160, algo=algo, name="tiny_blocks")
    res, states, status, _ = emu.replay(b, kf=256, kl=256, cf=4096, cl=16384, shape=6)
    check(b, res, states, status)
    assert int(states[0][0]) > 64, "the free blocks should span several chunks"


def test_ordered_random_small_heaps_and_partial_frees():
    rng = np.random.default_rng(13)
    parts = []
    for h in range(30):
        gran = int(rng.integers(1, 400))
        parts.append(W.random_tiny(int(rng.integers(1 << 30)), int(rng.integers(0, 400)),
                                   gran, align=int(1 << rng.integers(0, 12)),
                                   algo=int(rng.integers(0, 5)),
                                   max_granules=max(1, gran // int(rng.integers(1, 8))),
                                   p_partial=float(rng.uniform(0.0, 1.0))))
    b = W.concat(parts)
    res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=512, cl=512, shape=6)
    check(b, res, states, status)


def test_ordered_max_arena_edges_and_capacity():
    b = W.max_arena_batch()
    res, states, status, _ = emu.replay(b, kf=64, kl=64, cf=64, cl=192, shape=6)
    check(b, res, states, status)
    # at its capacities the ordered core refuses the same requests as the
    # lean core and ends in the same states
    b = W.concat([W.uniform_batch(seed=9, heaps=1, n=2500, algo=a) for a in ALGOS], "cap")
    r6, s6, st6, _ = emu.replay(b, kf=64, kl=64, cf=64, cl=192, shape=6)
    r3, s3, st3, _ = emu.replay(b, kf=64, kl=64, cf=64, cl=192, shape=3)
    assert (st3 == -4).all()
    assert np.array_equal(r6, r3) and np.array_equal(st6, st3)
    for h in range(b.heaps):
        assert np.array_equal(s6[h], s3[h])
