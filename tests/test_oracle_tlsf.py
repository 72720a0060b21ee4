"""Pins for the oracle's two-level segregated fit (TLSF, Sec. V-B): every
power of two split into 32 linear sub-classes, a good-fit request class, and
the segregated-fit list discipline.  Checked against the list model of
tests/models.py driven by an explicit table of class bounds (no bit
arithmetic, no bitmaps), against closed forms of the class function, and by
invariants after every step.  No GPU involved."""
import numpy as np
import pytest

import models
import oracle
from paper_2405_07079_amd import workloads as W
from test_oracle_partial import enumerate_partial
from test_oracle_pins import check_batch, check_invariants, oracle_state

TL = oracle.TLSF


def lower_bound(c):
    """Smallest byte size of class index c = fl * 32 + sl (may be fractional
    below 32 bytes; returned scaled by 32)."""
    fl, sl = divmod(c, 32)
    return (1 << fl) * (32 + sl)


def test_exhaustive_small_arena():
    # 128 granules of 16 B; sizes straddle sub-class boundaries of several
    # levels (16 B .. 2 KiB)
    cases = enumerate_partial(TL, 2048, 16, (16, 48, 80, 400, 1000, 2048), 4)
    assert len(cases) > 2_000
    check_batch(TL, 2048, 16, cases)


@pytest.mark.parametrize("granules,align,hi", ((64, 16, 1024), (4096, 64, 64 << 10),
                                               (1 << 14, 1, 4000)))
def test_random_traces_vs_model(granules, align, hi):
    rng = np.random.default_rng(3000 + granules + align)
    cases = []
    for _ in range(40):
        b = W.random_tiny(int(rng.integers(1 << 30)), 300, granules, align=align,
                          p_alloc=float(rng.uniform(0.45, 0.7)), algo=TL,
                          max_granules=max(1, hi // align), p_partial=0.3)
        m = models.make(TL, granules * align, align)
        res = models.replay(m, b.req.tolist())
        cases.append((b.req.tolist(), res, m.state()))
    check_batch(TL, granules * align, align, cases)


def test_class_bounds_closed_form():
    """A free block of exactly a class's lower bound sits in that class's
    list; one byte less sits in the class below it, or (below 32 B, where
    sub-classes are half bytes or finer) in the class of the last bound it
    reaches.  The heap's arena is the block itself, so it is the only free
    block."""
    for c in (5 * 32, 5 * 32 + 1, 6 * 32 + 17, 12 * 32 + 31, 20 * 32, 31 * 32 + 5):
        size = lower_bound(c) // 32
        below = max(k for k in range(c) if lower_bound(k) <= 32 * (size - 1))
        assert below == c - 1 or c == 5 * 32
        for s, want in ((size, c), (size - 1, below)):
            st = oracle_state(oracle.Heap(TL, s, 1))
            assert st["free"] == [(0, s)]
            where = [k for k, lst in enumerate(st["lists"]) if lst]
            assert where == [want], (s, where, want)
            assert st["bitmap"] == 1 << (want // 32)


def test_good_fit_request_class():
    """A request is served from the first non-empty class all of whose blocks
    are large enough.  At 1 KiB sub-classes are 32 B wide: a request of
    1040 B rounds up to class [1056, 1088), so a free 1048 B block, which
    would fit but shares class [1024, 1056) with smaller sizes, is passed
    over for a larger one; a request of 1024 B (a class bound) takes it."""
    h = oracle.Heap(TL, 1 << 16, 8)
    x = h.alloc(1048)            # [0, 1048)
    h.alloc(8)                   # separator
    y = h.alloc(2048)            # [1056, 3104)
    h.alloc(8)
    assert h.free(x) == 0 and h.free(y) == 0
    assert h.alloc(1040) == y
    assert h.alloc(1024) == x


def test_finer_than_segregated_fit():
    """Segregated fit serves 600 B from the 1024-2047 B class; TLSF from the
    sub-class just above 600 B, so it picks the 640 B block instead of the
    pushed-last 1536 B one."""
    def run(algo):
        h = oracle.Heap(algo, 1 << 16, 16)
        a = h.alloc(640)
        h.alloc(16)
        b = h.alloc(1536)
        h.alloc(16)
        h.free(a)
        h.free(b)               # pushed last
        return h.alloc(600), a, b
    r_sf, a_sf, b_sf = run(oracle.SEG_FIT)
    r_tl, a_tl, b_tl = run(TL)
    assert r_sf == b_sf          # class 10 = [1024, 2048): only the 1536 B block
    assert r_tl == a_tl          # sub-class of [608, 640) rounds up to [640, 672)


def test_invariants_every_step():
    A, g = 1 << 16, 16
    for seed in range(5):
        b = W.random_tiny(seed, 400, A // g, align=g, p_alloc=0.58, algo=TL,
                          max_granules=200)
        h = oracle.Heap(TL, A, g)
        for q in b.req:
            before = oracle_state(h)
            r = int(h.replay(np.array([q]))[0])
            st = oracle_state(h)
            check_invariants(st, TL, A, g)
            # every free block sits in the list of its class, once; first-level
            # bit fl set <=> one of lists fl*32 .. fl*32+31 non-empty
            where = {}
            for k, lst in enumerate(st["lists"]):
                for a in lst:
                    assert a not in where
                    where[a] = k
            assert sorted(where) == [a for a, _ in st["free"]]
            for a, s in st["free"]:
                c = where[a]
                assert lower_bound(c) <= 32 * s < lower_bound(c + 1)
            levels = {k // 32 for k, lst in enumerate(st["lists"]) if lst}
            assert st["bitmap"] == sum(1 << fl for fl in levels)
            if q >= 0 and r >= 0:
                s = max(g, -(-int(q) // g) * g)
                src = [(a, sz) for a, sz in before["free"] if a == r]
                assert len(src) == 1 and src[0][1] >= s
            elif q >= 0:
                assert before == st
