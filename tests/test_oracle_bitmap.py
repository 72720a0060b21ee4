"""Pins for the oracle's bitmask allocator with a next-fit search (Sec.
III-B): checked against the granule-bitmap model of tests/models.py, which
scans a literal list of free flags from the rover bit, and by invariants and
hand-made cases.  No GPU involved."""
import numpy as np
import pytest

import models
import oracle
from paper_2405_07079_amd import workloads as W
from test_oracle_partial import enumerate_partial
from test_oracle_pins import check_batch, check_invariants, oracle_state

BM = oracle.BITMAP


def test_exhaustive_small_arena():
    # 8 granules of 16 B; frees include partial ones (the victim keeps half,
    # or all but one granule)
    cases = enumerate_partial(BM, 128, 16, (16, 32, 48, 80, 128), 5)
    assert len(cases) > 10_000
    check_batch(BM, 128, 16, cases)


@pytest.mark.parametrize("granules,align", ((16, 16), (64, 16), (300, 1)))
def test_random_traces_vs_model(granules, align):
    rng = np.random.default_rng(4000 + granules)
    cases = []
    for _ in range(50):
        b = W.random_tiny(int(rng.integers(1 << 30)), 250, granules, align=align,
                          p_alloc=float(rng.uniform(0.45, 0.7)), algo=BM,
                          max_granules=max(1, granules // int(rng.integers(1, 6))),
                          p_partial=0.3)
        m = models.make(BM, granules * align, align)
        res = models.replay(m, b.req.tolist())
        cases.append((b.req.tolist(), res, m.state()))
    check_batch(BM, granules * align, align, cases)


def test_scan_starts_at_the_rover_not_the_block():
    """After [0, 32) is freed the whole arena is one free run, but the scan
    resumes at the rover (32): the list-based next fit takes the run's low
    end, the bitmask next fit the granules from the rover on."""
    for algo, want in ((oracle.NEXT_FIT, 0), (BM, 32)):
        h = oracle.Heap(algo, 256, 16)
        a = h.alloc(32)
        assert a == 0 and h.free(a) == 0
        assert h.alloc(32) == want
        st = oracle_state(h)
        assert st["rover"] == want + 32


def test_wraps_once():
    h = oracle.Heap(BM, 256, 16)
    xs = [h.alloc(64) for _ in range(4)]          # fills the arena; rover = 256
    assert xs == [0, 64, 128, 192]
    assert h.free(64) == 0
    assert h.alloc(32) == 64                      # nothing from 256 on: wrap
    assert h.alloc(48) == -1                      # 32 free granules, not 48 in a row
    assert oracle_state(h)["rover"] == 96


def test_invariants_every_step():
    A, g = 4096, 16
    for seed in range(6):
        b = W.random_tiny(seed, 400, A // g, align=g, p_alloc=0.58, algo=BM,
                          max_granules=40, p_partial=0.2)
        h = oracle.Heap(BM, A, g)
        for q in b.req:
            before = oracle_state(h)
            r = int(h.replay(np.array([q]))[0])
            st = oracle_state(h)
            check_invariants(st, BM, A, g)
            assert 0 <= st["rover"] <= A
            if q >= 0 and r >= 0:
                s = max(g, -(-int(q) // g) * g)
                assert st["rover"] == r + s
                # the run came out of one free block, at or after the old
                # rover if any such run existed
                src = [(a, sz) for a, sz in before["free"] if a <= r and r + s <= a + sz]
                assert len(src) == 1
                fits_after = any(max(a, before["rover"]) + s <= a + sz
                                 for a, sz in before["free"])
                assert (r >= before["rover"]) == fits_after
            elif q >= 0:
                assert before == st
