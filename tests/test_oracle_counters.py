"""Pins for the oracle's instrumentation counters (no GPU).

The oracle counts, per heap, the free-list entries a fit search inspects
(`examined`: first, next and best fit, the bitmask allocator) and the
segregated-fit records it reads or writes (`touched`: segregated fit and
TLSF).  The benchmark turns these counts into the metadata bytes the paper's
own structures would move per request, so both are pinned here, op by op,
against the brute-force models of tests/models.py, which share no code with
the oracle:

* first fit walks the address-ordered free list from its head to the first
  block that fits (Sec. II-A): it inspects (index of that block) + 1
  entries, or all of them when none fits;
* best fit walks the whole list, stopping early only at an exact size match
  (Alg. 3);
* next fit starts at the first block ending past the rover and walks the
  list cyclically to the first fit (Sec. II-A, Sec. IV);
* the bitmask allocator's first pass tries every free run from the rover on,
  its second pass every run from the start;
* segregated fit and TLSF touch only a bounded number of records per
  operation -- the constant-time allocation and coalescing the paper claims
  for the hash-table design (Sec. II-B, Sec. III-C, Sec. V-A) -- and the
  exact count follows from the list and neighbour shape before the
  operation: a pop or unlink touches the record and each list neighbour it
  relinks, a push the record and the old head, the used/free flip its
  record, and the adjacency fix-up the block after the changed one.
"""
import numpy as np
import pytest

import models
import oracle
from paper_2405_07079_amd import workloads as W

FF, NF, BF, SF, TLSF, BITMAP = 0, 1, 2, 3, 4, 5


def step_counts(algo, A, g, req):
    """Replay `req` one request at a time on an oracle heap and on the model;
    returns (per-request counter deltas, model predictions)."""
    h = oracle.Heap(algo, A, g)
    m = models.make(algo, A, g)
    got, want = [], []
    for q in req:
        q = int(q)
        want.append(predict(algo, m, q, A, g))
        e0, t0 = h.stats()
        r = int(h.replay(np.array([q], np.int64))[0])
        e1, t1 = h.stats()
        got.append((e1 - e0) if algo in (FF, NF, BF, BITMAP) else (t1 - t0))
        mr = models.replay(m, [q])[0]
        assert r == mr, (q, r, mr)
    return got, want


def predict(algo, m, q, A, g):
    """The counter delta the model's state implies for request q."""
    if algo in (FF, NF, BF, BITMAP):
        if q < 0:
            return 0                               # frees search nothing
        if q > A:
            return 0                               # rejected before any search
        s = models.granules(q, g)
        rs = models.runs(m.bits)                   # the free list, address order
        n = len(rs)
        if algo == FF:
            return next((i + 1 for i, (_, l) in enumerate(rs) if l >= s), n)
        if algo == BF:
            return next((i + 1 for i, (_, l) in enumerate(rs) if l == s), n)
        if algo == NF:
            if n == 0:
                return 0
            i0 = next((i for i, (a, l) in enumerate(rs) if a + l > m.rover), 0)
            for k in range(n):
                if rs[(i0 + k) % n][1] >= s:
                    return k + 1
            return n
        # bitmask: pass 1 from the rover, pass 2 from granule 0
        c1 = 0
        for a, l in rs:
            c1 += 1
            if max(a, m.rover) + s <= a + l:
                return c1
        return c1 + next((i + 1 for i, (_, l) in enumerate(rs) if l >= s), n)
    # segregated fit / TLSF: records touched
    blocks = m.blocks                               # [addr, size, free] by address

    def list_of(addr, size):
        return m.lists[m.cls(size)]

    def unlink_cost(addr, size):
        lst = list_of(addr, size)
        i = lst.index(addr)
        return 1 + (i > 0) + (i < len(lst) - 1)

    if q >= 0:
        if q > A:
            return 0
        s = models.granules(q, g) * g
        k = __import__("bisect").bisect_left(m.bounds, s * 32)
        c = next((c for c in range(k, len(m.lists)) if m.lists[c]), None)
        if c is None:
            return 0
        addr = m.lists[c][0]
        size = next(b[1] for b in blocks if b[0] == addr)
        n = 1 + (len(m.lists[c]) > 1) + 1          # pop the head, mark it used
        if size > s:
            rest = size - s
            c2 = m.cls(rest)
            head_left = len(m.lists[c2]) - (1 if c2 == c else 0)
            n += 1 + (head_left > 0)               # push the remainder
            n += (addr + size < A)                 # the next block's prev_adj
        return n
    if not m.live:
        return 0
    x = m.live[models.draw_index(q, len(m.live))]
    i = next(i for i, b in enumerate(blocks) if b[0] == x)
    size = blocks[i][1]
    n = 1 + (x > 0) + (x + size < A)               # the record and both neighbours
    end = x + size
    gone = []
    if i > 0 and blocks[i - 1][2]:
        n += unlink_cost(blocks[i - 1][0], blocks[i - 1][1])
        gone.append(blocks[i - 1])
    if i + 1 < len(blocks) and blocks[i + 1][2]:
        nb = blocks[i + 1]
        # unlinking the left block first can leave the right one's list
        # neighbour gone; count against the list as it then stands
        lst = [a for a in list_of(nb[0], nb[1])
               if not any(a == gb[0] for gb in gone)]
        j = lst.index(nb[0])
        n += 1 + (j > 0) + (j < len(lst) - 1)
        gone.append(nb)
        end = nb[0] + nb[1]
    n += (end < A)                                  # prev_adj of the block after
    start = gone[0][0] if gone and gone[0][0] < x else x
    merged = end - start
    lst = [a for a in list_of(start, merged) if not any(a == gb[0] for gb in gone)]
    n += 1 + (len(lst) > 0)                         # push the merged block
    return n


@pytest.mark.parametrize("algo", (FF, NF, BF, BITMAP))
@pytest.mark.parametrize("granules", (24, 64))
def test_fit_search_counts_entries_inspected(algo, granules):
    rng = np.random.default_rng(500 + algo * 3 + granules)
    for t in range(12):
        b = W.random_tiny(int(rng.integers(1 << 30)), 300, granules, align=16,
                          p_alloc=float(rng.uniform(0.5, 0.7)), algo=algo,
                          max_granules=max(1, granules // 6))
        got, want = step_counts(algo, granules * 16, 16, b.req)
        assert got == want


@pytest.mark.parametrize("algo", (SF, TLSF))
@pytest.mark.parametrize("granules", (24, 96))
def test_segregated_fit_records_touched(algo, granules):
    rng = np.random.default_rng(900 + algo * 5 + granules)
    for t in range(10):
        b = W.random_tiny(int(rng.integers(1 << 30)), 300, granules, align=16,
                          p_alloc=float(rng.uniform(0.5, 0.7)), algo=algo,
                          max_granules=max(1, granules // 8))
        got, want = step_counts(algo, granules * 16, 16, b.req)
        assert got == want


def per_request_touched(algo, b):
    h = oracle.Heap(algo, int(b.arena[0]), int(b.align[0]))
    out = []
    for q in b.req:
        t0 = h.stats()[1]
        h.replay(np.array([q], np.int64))
        out.append(h.stats()[1] - t0)
    return np.array(out), oracle.parse_state(h.state(), algo)


@pytest.mark.parametrize("algo", (SF, TLSF))
def test_segregated_fit_is_constant_time(algo):
    """Sec. II-B / V-A: segregated fit allocates and coalesces in constant
    time.  Per request the oracle touches at most 12 records (a free: the
    record, its two address neighbours, two unlinks of up to 3 records, the
    adjacency fix-up, a push of 2) and at most 6 for an allocation (pop 2,
    flag 1, push 2, fix-up 1), however many free blocks the heap holds: a
    heap with hundreds of free blocks costs no more per request than one
    with a handful."""
    small = W.random_tiny(3, 4000, 64, align=16, p_alloc=0.6, algo=algo, max_granules=8)
    big = W.uniform_batch(seed=2, heaps=1, n=20000, algo=algo)
    ts, ss = per_request_touched(algo, small)
    tb, sb = per_request_touched(algo, big)
    assert len(sb["free"]) >= 100 and len(ss["free"]) <= 16
    assert ts.max() <= 12 and tb.max() <= 12
    assert tb[big.req >= 0].max() <= 6 and ts[small.req >= 0].max() <= 6
    assert tb.mean() <= 8 and ts.mean() <= 8


def test_first_fit_examines_up_to_the_first_fit():
    """Hand-built heap: blocks of 1, 2, 3 and 4 granules freed apart from
    each other leave free holes of those sizes in address order; a request
    of 3 granules is served by the third hole after inspecting 3 entries, a
    request larger than every hole inspects all of them."""
    g = 16
    h = oracle.Heap(FF, 64 * g, g)
    offs = []
    for s in (1, 1, 2, 1, 3, 1, 4, 1):              # hole, separator, ...
        offs.append(h.alloc(s * g))
    for o in offs[0::2]:
        assert h.free(o) == 0
    # free list now: [0,1) [2,4) [5,8) [9,13) [14,64)
    e0 = h.stats()[0]
    assert h.alloc(3 * g) == 5 * g
    assert h.stats()[0] - e0 == 3
    e0 = h.stats()[0]
    assert h.alloc(60 * g) == -1                    # [5,8) is gone: 4 entries left
    assert h.stats()[0] - e0 == 4
