"""Pins for the CPU oracle: brute force, invariants, closed forms and the
statements the paper makes about its algorithms.  No GPU involved."""
import itertools

import numpy as np
import pytest

import oracle
import models
from paper_2405_07079_amd import workloads as W

FF, NF, BF, SF = 0, 1, 2, 3
ALGOS = (FF, NF, BF, SF)


def oracle_state(h):
    return oracle.parse_state(h.state(), h.algo)


def same_state(a, b, algo):
    assert a["free"] == b["free"]
    assert a["live"] == b["live"]
    assert a["rover"] == b["rover"]
    if algo == SF:
        assert a["bitmap"] == b["bitmap"]
        assert [list(x) for x in a["lists"]] == [list(x) for x in b["lists"]]


# ---------------------------------------------------------------------------
# Exhaustive enumeration against the brute-force models
# ---------------------------------------------------------------------------

def enumerate_traces(algo, arena, align, sizes, depth):
    """Every request sequence up to `depth` over: alloc of each size in
    `sizes`, and free of each live block (or a free with nothing live).
    Yields (trace, model results, model state)."""
    out = []

    def visit(seq):
        m = models.make(algo, arena, align)
        res = models.replay(m, seq)
        out.append((list(seq), res, m.state()))
        if len(seq) == depth:
            return
        L = len(m.live)
        ops = list(sizes) + ([models.draw_for(i, L) for i in range(L)] if L else [-1])
        for op in ops:
            visit(seq + [op])

    visit([])
    return out


def check_batch(algo, arena, align, cases):
    lens = np.array([len(c[0]) for c in cases], np.int64)
    off = np.zeros(len(cases) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    req = np.array([q for c in cases for q in c[0]], np.int64)
    b = W.Batch("enum", np.full(len(cases), arena, np.int64),
                np.full(len(cases), align, np.int64),
                np.full(len(cases), algo, np.int32), off, req)
    res, states, _ = oracle.replay_batch(b, threads=4)
    for i, (seq, mres, mstate) in enumerate(cases):
        got = res[off[i]:off[i + 1]].tolist()
        assert got == mres, (algo, seq, got, mres)
        same_state(oracle.parse_state(states[i], algo), mstate, algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_exhaustive_depth5(algo):
    # 6-granule arena of 16 B granules; sizes cover 0 B, exact and ragged
    # multiples, the whole arena and one byte past it.
    cases = enumerate_traces(algo, 96, 16, (0, 16, 17, 48, 64, 96, 97), 5)
    assert len(cases) > 10_000
    check_batch(algo, 96, 16, cases)


@pytest.mark.parametrize("algo", ALGOS)
def test_exhaustive_depth6_small_sizes(algo):
    # 8-granule arena, a denser size alphabet that keeps many blocks live.
    cases = enumerate_traces(algo, 128, 16, (16, 32, 48), 6)
    check_batch(algo, 128, 16, cases)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("granules", (16, 37, 64))
def test_random_traces_vs_models(algo, granules):
    rng = np.random.default_rng(1000 + 7 * algo + granules)
    cases = []
    for t in range(60):
        b = W.random_tiny(int(rng.integers(1 << 30)), 250, granules, align=16,
                          p_alloc=float(rng.uniform(0.45, 0.7)), algo=algo)
        m = models.make(algo, granules * 16, 16)
        res = models.replay(m, b.req.tolist())
        cases.append((b.req.tolist(), res, m.state()))
    check_batch(algo, granules * 16, 16, cases)


# ---------------------------------------------------------------------------
# Invariants after every operation
# ---------------------------------------------------------------------------

def check_invariants(st, algo, A, g):
    free, live = st["free"], st["live"]
    blocks = sorted([(a, s, True) for a, s in free] + [(a, s, False) for a, s in live])
    # I2: alignment
    assert all(a % g == 0 and s % g == 0 and s > 0 for a, s, _ in blocks)
    # I1: the blocks tile [0, A) exactly (disjoint, conservation)
    pos = 0
    for a, s, _ in blocks:
        assert a == pos
        pos += s
    assert pos == A
    # I3: no two free blocks adjacent
    for (a, s, f), (a2, s2, f2) in zip(blocks, blocks[1:]):
        assert not (f and f2)
    assert free == sorted(free)
    if algo == NF:
        assert 0 <= st["rover"] <= A
    if algo == SF:
        # I4: every free block sits in the list of floor(log2 size), once;
        # bit k set <=> list k non-empty.
        where = {}
        for k, lst in enumerate(st["lists"]):
            assert bool(st["bitmap"] >> k & 1) == bool(len(lst))
            for a in lst:
                assert a not in where
                where[a] = k
        assert sorted(where) == [a for a, _ in free]
        for a, s in free:
            assert 2 ** where[a] <= s < 2 ** (where[a] + 1)


@pytest.mark.parametrize("algo", ALGOS)
def test_invariants_every_step(algo):
    A, g = 4096, 16
    for seed in range(6):
        b = W.random_tiny(seed, 400, A // g, align=g, p_alloc=0.58, algo=algo,
                          max_granules=40)
        h = oracle.Heap(algo, A, g)
        for q in b.req:
            before = oracle_state(h)
            r = int(h.replay(np.array([q]))[0])
            st = oracle_state(h)
            check_invariants(st, algo, A, g)
            if q >= 0:
                s = max(g, -(-int(q) // g) * g)
                mx = max([sz for _, sz in before["free"]], default=0)
                if algo == SF:
                    need = 1 << (s - 1).bit_length()
                    # I5/I6: fails iff no free block reaches 2^ceil(log2 s)
                    assert (r == -1) == (mx < need)
                else:
                    assert (r == -1) == (mx < s)
                if r >= 0:
                    # taken from the low end of a free block that holds s
                    src = [(a, sz) for a, sz in before["free"] if a == r]
                    assert len(src) == 1 and src[0][1] >= s
                    assert (r, s) == st["live"][-1]
                else:
                    assert before == st, "a failed allocation changed the state"


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("algo", ALGOS)
def test_alloc_only_is_prefix_sum(algo):
    """With only allocations the free space is one block at the top; every
    success is placed at the running total of the successful sizes."""
    A, g = 1 << 20, 64
    rng = np.random.default_rng(algo)
    h = oracle.Heap(algo, A, g)
    top = 0
    for req in rng.integers(0, 40_000, 300):
        s = max(g, -(-int(req) // g) * g)
        r = h.alloc(int(req))
        remaining = A - top
        ok = remaining >= ((1 << (s - 1).bit_length()) if algo == SF else s)
        if ok:
            assert r == top
            top += s
        else:
            assert r == -1


@pytest.mark.parametrize("algo", ALGOS)
def test_free_everything_restores_initial_state(algo):
    A, g = 1 << 16, 16
    for seed in range(5):
        b = W.random_tiny(seed, 500, A // g, align=g, algo=algo, max_granules=100)
        h = oracle.Heap(algo, A, g)
        h.replay(b.req)
        live = [a for a, _ in oracle_state(h)["live"]]
        order = np.random.default_rng(seed).permutation(len(live))
        for i in order:
            assert h.free(live[i]) == 0
        st = oracle_state(h)
        assert st["free"] == [(0, A)] and st["live"] == []
        if algo == SF:
            k = A.bit_length() - 1
            assert st["bitmap"] == 1 << k and st["lists"][k] == [0]


def test_first_fit_lifo_is_bump_allocator():
    """Freeing in reverse allocation order under first fit rolls a bump
    pointer back: every allocation lands at the current top."""
    A, g = 1 << 16, 16
    rng = np.random.default_rng(5)
    h = oracle.Heap(FF, A, g)
    stack, top = [], 0
    for _ in range(2000):
        if stack and rng.random() < 0.45:
            a, s = stack.pop()
            assert h.free(a) == 0
            top = a
        else:
            s = max(g, -(-int(rng.integers(1, 2000)) // g) * g)
            r = h.alloc(s)
            if top + s <= A:
                assert r == top
                stack.append((r, s))
                top += s
            else:
                assert r == -1


@pytest.mark.parametrize("algo", ALGOS)
def test_whole_arena_alternates(algo):
    h = oracle.Heap(algo, 1 << 12, 16)
    assert h.alloc(1 << 12) == 0
    assert h.alloc(0) == -1
    assert h.free(0) == 0
    assert h.alloc(1 << 12) == 0
    assert h.alloc(1 << 12) == -1


# ---------------------------------------------------------------------------
# Statements of the paper
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("algo", ALGOS)
def test_initial_state_single_block(algo):
    """Alg. 6: the free list starts as the single block holding the heap."""
    A = 3 << 20
    st = oracle_state(oracle.Heap(algo, A, 4096))
    assert st["free"] == [(0, A)] and st["live"] == []
    if algo == SF:
        assert st["bitmap"] == 1 << 21 and st["lists"][21] == [0]


@pytest.mark.parametrize("algo", ALGOS)
def test_low_end_split(algo):
    """Alg. 1 / Alg. 4: the block is cut from the low end of the free block."""
    h = oracle.Heap(algo, 1 << 12, 16)
    assert h.alloc(100) == 0           # 112 bytes taken from [0, 4096)
    st = oracle_state(h)
    assert st["free"] == [(112, 4096 - 112)]
    assert st["live"] == [(0, 112)]


def test_seg_fit_nearly_four_times():
    """Sec. V-A: the selected block may be nearly 4x the request -- a request
    just above 2^(k-1) is served from class k, whose blocks are below 2^(k+1).
    The class is the 0-based ceil(log2 s); the block class k-1 is never used
    for it even when a block there would fit."""
    g = 16
    h = oracle.Heap(SF, 1 << 16, g)
    # carve [0,1008) | [1008,2032) | rest, then free the first two separately
    a = h.alloc(1008)                  # 1008 B  -> class 9 block once freed
    b = h.alloc(16)                    # separator
    c = h.alloc(2032)                  # 2032 B  -> class 10 block once freed
    d = h.alloc(16)
    assert (a, b, c, d) == (0, 1008, 1024, 3056)
    assert h.free(a) == 0 and h.free(c) == 0
    st = oracle_state(h)
    assert st["lists"][9] == [0] and st["lists"][10] == [1024]
    # request 528 B: ceil(log2 528) = 10 -> class 10, a 2032 B block (3.85x),
    # although the 1008 B class-9 block would fit.
    r = h.alloc(528)
    assert r == 1024
    assert 2032 / 528 > 3.8 and 2032 / 528 < 4
    # a 1-based class index (ffs) would have used class 11 and failed here,
    # or taken the top block; an off-by-one downwards would have taken 0.


def test_seg_fit_lifo_lists():
    """Alg. 4 / Alg. 5: lists are popped and pushed at the head."""
    g = 16
    h = oracle.Heap(SF, 1 << 16, g)
    offs = [h.alloc(256) for _ in range(6)]        # 6 x 256 B, then the rest
    assert offs == [256 * i for i in range(6)]
    # free blocks 0, 2, 4 (non-adjacent): each is a 256 B class-8 block
    for i in (0, 2, 4):
        assert h.free(offs[i]) == 0
    st = oracle_state(h)
    assert st["lists"][8] == [1024, 512, 0]        # last pushed first
    assert h.alloc(200) == 1024                    # head popped
    assert oracle_state(h)["lists"][8] == [512, 0]


def test_seg_fit_merge_pushes_at_head():
    g = 16
    h = oracle.Heap(SF, 1 << 12, g)
    offs = [h.alloc(256) for _ in range(4)]
    assert h.free(offs[0]) == 0                    # [0,256) class 8
    assert h.free(offs[2]) == 0                    # [512,768) class 8
    st = oracle_state(h)
    assert st["lists"][8] == [512, 0]
    assert h.free(offs[1]) == 0                    # merges all three: 768 B, class 9
    st = oracle_state(h)
    assert st["lists"][8] == [] and st["lists"][9] == [0]
    assert st["free"][0] == (0, 768)


def test_best_fit_exact_and_ties():
    """Sec. II-A: best fit takes the smallest block that fits; an exact size
    match ends the search; equal sizes go to the lowest address."""
    g = 16
    h = oracle.Heap(BF, 1 << 12, g)
    offs = [h.alloc(s) for s in (64, 16, 128, 16, 64, 16, 96, 16)]
    for i in (0, 2, 4, 6):
        assert h.free(offs[i]) == 0
    # free: [0,64) [80,208) [224,288) [304,400) + tail
    assert h.alloc(64) == 0            # exact, lowest address of the two 64s
    assert h.alloc(64) == 224
    assert h.alloc(90) == 304          # 96 is the smallest >= 96
    assert h.alloc(100) == 80          # 128 block


def test_first_fit_lowest_address():
    g = 16
    h = oracle.Heap(FF, 1 << 12, g)
    offs = [h.alloc(s) for s in (32, 16, 128, 16)]
    h.free(offs[0]); h.free(offs[2])
    # free: [0,32) [48,176) [192,4096)
    assert h.alloc(48) == 48
    assert h.alloc(32) == 0
    assert h.alloc(80) == 96


def test_next_fit_resumes_at_rover():
    """Sec. II-A / Sec. IV: next fit resumes where the previous search ended
    and wraps around to the lowest address."""
    g = 16
    h = oracle.Heap(NF, 256, g)
    offs = [h.alloc(32) for _ in range(8)]         # fills 256 B
    assert offs == [32 * i for i in range(8)]
    assert oracle_state(h)["rover"] == 256
    h.free(32); h.free(128)                        # holes at 32 and 128
    assert h.alloc(16) == 32                       # wraps to the lowest hole
    assert oracle_state(h)["rover"] == 48
    assert h.alloc(16) == 48                       # continues in the same hole
    assert h.alloc(16) == 128                      # next hole, not back to 32
    h.free(32)                                     # hole [32,48) behind rover
    assert h.alloc(32) == -1                       # nothing of 32 B anywhere
    assert oracle_state(h)["rover"] == 144         # unchanged by failure


# ---------------------------------------------------------------------------
# Argument handling
# ---------------------------------------------------------------------------

def test_bad_params_rejected():
    for algo, A, g in ((6, 1024, 16), (0, 1024, 24), (0, 1000, 16), (0, 0, 16),
                       (0, 1 << 36, 16)):
        with pytest.raises(ValueError):
            oracle.Heap(algo, A, g)


@pytest.mark.parametrize("algo", ALGOS)
def test_bad_free_keeps_state(algo):
    h = oracle.Heap(algo, 1 << 12, 16)
    a = h.alloc(64)
    h.alloc(64)
    before = h.state().tolist()
    assert h.free(a + 16) == oracle.E_BADFREE      # inside a block
    assert h.free(4000) == oracle.E_BADFREE        # in free space
    assert h.free(a) == 0
    after = h.state().tolist()
    assert h.free(a) == oracle.E_BADFREE           # double free
    assert h.state().tolist() == after
    assert before != after


@pytest.mark.parametrize("algo", ALGOS)
def test_free_with_nothing_live(algo):
    h = oracle.Heap(algo, 1 << 12, 16)
    res = h.replay(np.array([-1, -5, 100, -1, -7], np.int64))
    assert res.tolist() == [-1, -1, 0, 0, -1]
