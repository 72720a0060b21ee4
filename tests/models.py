"""Brute-force allocator models used to pin the oracle.

They share nothing with the oracle's code and use different representations:

* Sequential fits run on a granule bitmap -- the bitmask representation of
  Sec. III-B (one flag per smallest allocatable unit, allocation = finding a
  run of free flags, free = setting the flags back so coalescing is
  implicit).  The free list is then, by construction, the set of maximal free
  runs, and first/next/best fit are stated directly on those runs.
* Segregated fit keeps a Python list of all blocks (address, size, free) and
  64 plain Python lists as the class lists (head at index 0); neighbours are
  found by scanning the block list by address instead of following links.
  TLSF is the same model over 64 x 32 classes given by an explicit sorted
  table of class lower bounds (2^fl + sl * 2^fl / 32): a block belongs to the
  last class whose bound it reaches, a request takes the first non-empty
  class whose bound is at least its size -- bisection instead of the bit
  arithmetic and two-level bitmaps of the oracle.

Both are O(arena) per operation and meant for tiny heaps only.
"""
from __future__ import annotations

import bisect

FIRST_FIT, NEXT_FIT, BEST_FIT, SEG_FIT, TLSF, BITMAP = 0, 1, 2, 3, 4, 5

# class lower bounds, scaled by 32 so that the TLSF ones are integers
SF_BOUNDS = [(1 << k) * 32 for k in range(64)]
TLSF_BOUNDS = [(1 << fl) * (32 + sl) for fl in range(64) for sl in range(32)]


def granules(req: int, g: int) -> int:
    """Size in granules: at least one granule, rounded up (division form)."""
    return max(1, -(-req // g))


def runs(bits):
    """Maximal runs of free flags as (start, length), address order."""
    out, i, n = [], 0, len(bits)
    while i < n:
        if bits[i]:
            j = i
            while j < n and bits[j]:
                j += 1
            out.append((i, j - i))
            i = j
        else:
            i += 1
    return out


class BitmapHeap:
    """First / next / best fit on a granule bitmap (True = free)."""

    def __init__(self, algo: int, arena: int, align: int):
        assert algo in (FIRST_FIT, NEXT_FIT, BEST_FIT, BITMAP)
        self.algo, self.g, self.n = algo, align, arena // align
        self.bits = [True] * self.n
        self.rover = 0                   # granule index
        self.used = {}                   # granule start -> granules
        self.live = []                   # replay-driver order

    def alloc(self, req: int) -> int:
        if req > self.n * self.g:
            return -1
        s = granules(req, self.g)
        if self.algo == BITMAP:
            # Sec. III-B with a next-fit search: the first s free flags in a
            # row, scanning from the rover bit, then from bit 0
            starts = list(range(self.rover, self.n - s + 1)) + list(range(0, self.n - s + 1))
            a = next((p for p in starts if all(self.bits[p:p + s])), None)
            if a is None:
                return -1
            for i in range(a, a + s):
                self.bits[i] = False
            self.rover = a + s
            self.used[a] = s
            self.live.append(a * self.g)
            return a * self.g
        fits = [(a, l) for a, l in runs(self.bits) if l >= s]
        if not fits:
            return -1
        if self.algo == FIRST_FIT:
            a, _ = fits[0]
        elif self.algo == BEST_FIT:
            a, _ = min(fits, key=lambda r: (r[1], r[0]))
        else:
            # cyclic order starting at the first run whose end is past the rover
            after = [r for r in fits if r[0] + r[1] > self.rover]
            a, _ = (after or fits)[0]
        for i in range(a, a + s):
            self.bits[i] = False
        if self.algo == NEXT_FIT:
            self.rover = a + s
        self.used[a] = s
        self.live.append(a * self.g)
        return a * self.g

    def free(self, off: int) -> int:
        a = off // self.g
        if off % self.g or a not in self.used:
            return -3
        s = self.used.pop(a)
        i = self.live.index(off)
        self.live[i] = self.live[-1]
        self.live.pop()
        for k in range(a, a + s):
            self.bits[k] = True
        return 0

    def free_partial(self, off: int) -> int:
        """Free [off, end of the used block holding off): the used block keeps
        its head (Sec. II-A); at the block's start this is a whole free."""
        if off % self.g:
            return -3
        x = off // self.g
        holder = [a for a, s in self.used.items() if a <= x < a + s]
        if not holder:
            return -3
        a = holder[0]
        if a == x:
            return self.free(off)
        end = a + self.used[a]
        self.used[a] = x - a
        for k in range(x, end):
            self.bits[k] = True
        return 0

    def state(self):
        g = self.g
        return dict(free=[(a * g, l * g) for a, l in runs(self.bits)],
                    live=[(a, self.used[a // g] * g) for a in self.live],
                    rover=self.rover * g if self.algo in (NEXT_FIT, BITMAP) else -1,
                    bitmap=0, lists=None)


class ListSegFit:
    """Segregated fit with a flat block list and 64 Python class lists."""

    def __init__(self, arena: int, align: int, bounds=SF_BOUNDS):
        self.A, self.g, self.bounds = arena, align, bounds
        self.blocks = [[0, arena, True]]          # [addr, size, free], by address
        self.lists = [[] for _ in bounds]         # addresses, head first
        self.lists[self.cls(arena)].insert(0, 0)
        self.live = []

    def cls(self, size: int) -> int:              # last class whose bound size reaches
        return bisect.bisect_right(self.bounds, size * 32) - 1

    def _find(self, addr):
        for i, b in enumerate(self.blocks):
            if b[0] == addr:
                return i
        return None

    def alloc(self, req: int) -> int:
        if req > self.A:
            return -1
        s = granules(req, self.g) * self.g
        k = bisect.bisect_left(self.bounds, s * 32)   # first class whose bound is >= s
        c = next((c for c in range(k, len(self.lists)) if self.lists[c]), None)
        if c is None:
            return -1
        addr = self.lists[c].pop(0)
        i = self._find(addr)
        blk = self.blocks[i]
        blk[2] = False
        if blk[1] > s:
            rest = [addr + s, blk[1] - s, True]
            blk[1] = s
            self.blocks.insert(i + 1, rest)
            self.lists[self.cls(rest[1])].insert(0, rest[0])
        self.live.append(addr)
        return addr

    def free(self, off: int) -> int:
        i = self._find(off)
        if i is None or self.blocks[i][2]:
            return -3
        j = self.live.index(off)
        self.live[j] = self.live[-1]
        self.live.pop()
        start, size = self.blocks[i][0], self.blocks[i][1]
        lo, hi = i, i
        if i > 0 and self.blocks[i - 1][2]:
            left = self.blocks[i - 1]
            self.lists[self.cls(left[1])].remove(left[0])
            start, size, lo = left[0], size + left[1], i - 1
        if i + 1 < len(self.blocks) and self.blocks[i + 1][2]:
            right = self.blocks[i + 1]
            self.lists[self.cls(right[1])].remove(right[0])
            size, hi = size + right[1], i + 1
        self.blocks[lo:hi + 1] = [[start, size, True]]
        self.lists[self.cls(size)].insert(0, start)
        return 0

    def free_partial(self, off: int) -> int:
        """Segregated fit frees whole keyed blocks only."""
        return self.free(off)

    def state(self):
        sizes = {b[0]: b[1] for b in self.blocks}
        bitmap = 0
        per_bit = len(self.lists) // 64           # TLSF: a bit per first level
        for c in range(len(self.lists)):
            if self.lists[c]:
                bitmap |= 1 << (c // per_bit)
        return dict(free=[(b[0], b[1]) for b in self.blocks if b[2]],
                    live=[(a, sizes[a]) for a in self.live],
                    rover=-1, bitmap=bitmap, lists=[list(l) for l in self.lists])


def make(algo: int, arena: int, align: int):
    if algo == SEG_FIT:
        return ListSegFit(arena, align)
    if algo == TLSF:
        return ListSegFit(arena, align, TLSF_BOUNDS)
    return BitmapHeap(algo, arena, align)


def draw_index(q: int, n_live: int) -> int:
    """The replay driver's choice of live entry for a free request."""
    r = (~q) & 0xFFFFFFFF
    return (r * n_live) >> 32


def draw_for(index: int, n_live: int) -> int:
    """An encoded free request whose draw selects live[index] of n_live."""
    r = (index * (1 << 32) + n_live - 1) // n_live
    return -(r + 1)


def draw_cut(q: int) -> int:
    """The 31-bit cut of an encoded free request (0: free the whole block)."""
    return (~q) >> 32


def free_request(draw: int, cut: int = 0) -> int:
    """Encode a free request from its 32-bit draw and 31-bit cut."""
    assert 0 <= draw < (1 << 32) and 0 <= cut < (1 << 31)
    return -((cut << 32 | draw) + 1)


def replay(model, req):
    """Replay an encoded trace on a model; returns the result list.  A free
    keeps the victim's first floor(cut * granules / 2^31) granules live on
    the sequential fits (none on segregated fit) and frees the rest."""
    out = []
    for q in req:
        q = int(q)
        if q >= 0:
            out.append(model.alloc(q))
        elif not model.live:
            out.append(-1)
        else:
            i = draw_index(q, len(model.live))
            off = model.live[i]
            keep = 0
            if isinstance(model, BitmapHeap):
                keep = (draw_cut(q) * model.used[off // model.g]) >> 31
            if keep:
                assert model.free_partial(off + keep * model.g) == 0
                out.append(off + keep * model.g)
            else:
                assert model.free(off) == 0
                out.append(off)
    return out
