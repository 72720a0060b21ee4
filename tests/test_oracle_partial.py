"""Pins for the oracle's partial deallocation (Sec. II-A, Alg. 2): freeing an
address inside a live block keeps the block's head live and frees its tail.
Checked against the granule-bitmap model (tests/models.py), where a partial
free just sets the tail's flags, and against the paper's own example.  No GPU
involved."""
import numpy as np
import pytest

import models
import oracle
from paper_2405_07079_amd import workloads as W
from test_oracle_pins import check_batch, check_invariants, oracle_state

FF, NF, BF, SF = 0, 1, 2, 3
SEQ = (FF, NF, BF)
CUTS = (0, 1 << 30, (1 << 31) - 1)   # whole block, keep half, keep all but one granule


def enumerate_partial(algo, arena, align, sizes, depth):
    """Every request sequence up to `depth` over: alloc of each size, and a
    free of each live block with each cut in CUTS."""
    out = []

    def visit(seq):
        m = models.make(algo, arena, align)
        res = models.replay(m, seq)
        out.append((list(seq), res, m.state()))
        if len(seq) == depth:
            return
        L = len(m.live)
        frees = []
        for i in range(L):
            draw = ~models.draw_for(i, L)
            frees += [models.free_request(draw, c) for c in CUTS]
        for op in list(sizes) + (frees or [-1]):
            visit(seq + [op])

    visit([])
    return out


@pytest.mark.parametrize("algo", (FF, NF, BF, SF))
def test_exhaustive_partial_depth5(algo):
    # 6-granule arena of 16 B granules; blocks of 1-6 granules are cut at
    # floor(s/2) and s-1 granules.  Segregated fit ignores the cut.
    cases = enumerate_partial(algo, 96, 16, (16, 32, 64, 96), 5)
    assert len(cases) > 5_000
    check_batch(algo, 96, 16, cases)


@pytest.mark.parametrize("algo", (FF, NF, BF, SF))
@pytest.mark.parametrize("granules", (16, 64))
def test_random_partial_traces_vs_models(algo, granules):
    rng = np.random.default_rng(2000 + 7 * algo + granules)
    cases = []
    for _ in range(60):
        b = W.random_tiny(int(rng.integers(1 << 30)), 250, granules, align=16,
                          p_alloc=float(rng.uniform(0.45, 0.7)), algo=algo,
                          p_partial=float(rng.uniform(0.2, 0.9)))
        m = models.make(algo, granules * 16, 16)
        res = models.replay(m, b.req.tolist())
        cases.append((b.req.tolist(), res, m.state()))
    check_batch(algo, granules * 16, 16, cases)


@pytest.mark.parametrize("algo", SEQ)
def test_paper_example_last_2kB_of_10kB(algo):
    """Sec. II-A: freeing the last 2 kB of a 10 kB block shrinks the block to
    8 kB and frees those 2 kB (here beside a live block, so they stay a free
    block of their own)."""
    h = oracle.Heap(algo, 64 * 1024, 1024)
    a = h.alloc(10 * 1024)
    b = h.alloc(1024)
    assert (a, b) == (0, 10 * 1024)
    assert h.free_partial(8 * 1024) == 0
    st = oracle_state(h)
    assert st["live"] == [(0, 8 * 1024), (10 * 1024, 1024)]
    assert st["free"] == [(8 * 1024, 2 * 1024), (11 * 1024, 53 * 1024)]


@pytest.mark.parametrize("algo", SEQ)
def test_partial_tail_merges_with_free_successor(algo):
    h = oracle.Heap(algo, 16 * 1024, 1024)
    a = h.alloc(4 * 1024)            # [0, 4k); the rest of the arena is free
    assert h.free_partial(a + 1024) == 0
    st = oracle_state(h)
    assert st["live"] == [(0, 1024)]
    assert st["free"] == [(1024, 15 * 1024)]


@pytest.mark.parametrize("algo", SEQ)
def test_partial_free_errors_keep_state(algo):
    h = oracle.Heap(algo, 1 << 12, 16)
    a = h.alloc(256)
    h.alloc(64)
    before = h.state().tolist()
    assert h.free_partial(a + 8) == oracle.E_BADFREE       # not a granule boundary
    assert h.free_partial(3000) == oracle.E_BADFREE        # in free space
    assert h.free_partial(-16) == oracle.E_BADFREE
    assert h.free_partial(1 << 12) == oracle.E_BADFREE
    assert h.state().tolist() == before
    assert h.free_partial(a + 64) == 0                     # interior: tail freed
    assert oracle_state(h)["live"][0] == (a, 64)
    assert h.free_partial(a + 64) == oracle.E_BADFREE      # now in free space
    assert h.free_partial(a) == 0                          # the head: whole free
    assert [x for x, _ in oracle_state(h)["live"]] == [256]


def test_seg_fit_interior_address_is_a_bad_free():
    h = oracle.Heap(SF, 1 << 12, 16)
    a = h.alloc(256)
    before = h.state().tolist()
    assert h.free_partial(a + 64) == oracle.E_BADFREE
    assert h.state().tolist() == before
    assert h.free_partial(a) == 0


@pytest.mark.parametrize("algo", SEQ)
def test_partial_replay_invariants_every_step(algo):
    A, g = 4096, 16
    for seed in range(4):
        b = W.random_tiny(seed, 300, A // g, align=g, p_alloc=0.58, algo=algo,
                          max_granules=40, p_partial=0.6)
        h = oracle.Heap(algo, A, g)
        for q in b.req:
            before = oracle_state(h)
            r = int(h.replay(np.array([q]))[0])
            st = oracle_state(h)
            check_invariants(st, algo, A, g)
            if q < 0 and before["live"]:
                live = dict(before["live"])
                keep = r - max(x for x in live if x <= r)
                # the victim keeps exactly `keep` bytes; the live count drops
                # only for a whole free
                assert len(st["live"]) == len(before["live"]) - (keep == 0)
                if keep:
                    assert dict(st["live"])[r - keep] == keep
