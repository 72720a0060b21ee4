"""Seeded synthetic request streams for allocator replay.

This module only draws random numbers and lays them out; it holds none of the
allocator's arithmetic (no size rounding, no fit choice, no coalescing).  It is
the one piece of code shared by the GPU path and by the CPU checker.

Request encoding (one int64 per request, per heap):

* ``req >= 0`` -- allocate ``req`` bytes (the raw size as drawn; the allocator
  normalises it to its alignment).
* ``req <  0`` -- free one live block.  ``r = -req - 1`` is a uniform 32-bit
  draw made by the workload; the replay engine maps it to an index into its
  list of live blocks (blocks returned by a successful allocation and not yet
  freed), so "free a uniformly chosen live block" needs no knowledge of the
  allocator's outcomes at generation time.

A batch is a CSR layout: heap ``h`` owns ``req[req_off[h]:req_off[h+1]]``, with
per-heap arena size (bytes), alignment (bytes, a power of two) and algorithm.

Every heap draws from its own stream ``PCG64(SeedSequence(seed,
spawn_key=(h,)))``, so any single heap of a large batch can be regenerated on
its own.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

FIRST_FIT, NEXT_FIT, BEST_FIT, SEG_FIT, TLSF = 0, 1, 2, 3, 4
ALGO_NAMES = {FIRST_FIT: "first_fit", NEXT_FIT: "next_fit",
              BEST_FIT: "best_fit", SEG_FIT: "seg_fit", TLSF: "tlsf"}

# the bitmask allocator (Sec. III-B) has its own replay entry point and is
# not among the algorithms above, which the table-based replay serves
BITMAP = 5

KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30


@dataclass
class Batch:
    """A batch of independent heaps and their request streams (CSR)."""
    name: str
    arena: np.ndarray      # int64 [H], bytes
    align: np.ndarray      # int64 [H], bytes, power of two
    algo: np.ndarray       # int32 [H]
    req_off: np.ndarray    # int64 [H+1]
    req: np.ndarray        # int64 [N]
    meta: dict = field(default_factory=dict)

    @property
    def heaps(self) -> int:
        return int(self.arena.shape[0])

    @property
    def requests(self) -> int:
        return int(self.req.shape[0])

    def heap_trace(self, h: int) -> np.ndarray:
        return self.req[self.req_off[h]:self.req_off[h + 1]]

    def with_algo(self, algo: int) -> "Batch":
        """Same streams, every heap switched to ``algo``."""
        name = ALGO_NAMES.get(algo, "bitmap" if algo == BITMAP else str(algo))
        return Batch(f"{self.name}/{name}", self.arena, self.align,
                     np.full_like(self.algo, algo), self.req_off, self.req,
                     dict(self.meta))

    def subset(self, heaps) -> "Batch":
        """A batch holding only the listed heaps, in the listed order."""
        heaps = np.asarray(heaps, dtype=np.int64)
        lens = self.req_off[heaps + 1] - self.req_off[heaps]
        off = np.zeros(len(heaps) + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        req = np.concatenate([self.heap_trace(int(h)) for h in heaps]) \
            if len(heaps) else np.zeros(0, np.int64)
        return Batch(f"{self.name}[{len(heaps)}]", self.arena[heaps].copy(),
                     self.align[heaps].copy(), self.algo[heaps].copy(), off,
                     req, dict(self.meta))


def heap_rng(seed: int, h: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence(entropy=seed, spawn_key=(h,))))


def log_uniform_int(rng: np.random.Generator, n: int, lo: float, hi,
                    ) -> np.ndarray:
    """floor(exp(ln lo + u ln(hi/lo))) clamped to [lo, hi]; ``hi`` may be an
    array (per element upper bound)."""
    u = rng.random(n)
    hi = np.asarray(hi, dtype=np.float64)
    v = np.floor(np.exp(np.log(lo) + u * np.log(hi / lo)))
    return np.clip(v, lo, hi).astype(np.int64)


def _stream(rng: np.random.Generator, n: int, p_alloc: float, sizes: np.ndarray,
            p_partial: float = 0.0) -> np.ndarray:
    """Mix allocation sizes with free draws: step i allocates w.p. p_alloc.
    A free is encoded as -(u + 1) with u = cut << 32 | draw: a uniform 32-bit
    draw picks the victim, and w.p. p_partial a cut uniform on [1, 2^31)
    keeps that fraction of the victim live (partial deallocation; the cut is
    0 otherwise, and no numbers are drawn for it when p_partial is 0)."""
    dec = rng.random(n)
    draw = rng.integers(0, 1 << 32, n, dtype=np.int64)
    if p_partial > 0.0:
        part = rng.random(n) < p_partial
        cut = rng.integers(1, 1 << 31, n, dtype=np.int64)
        draw = draw | np.where(part, cut, 0) << 32
    return np.where(dec < p_alloc, sizes, -(draw + 1)).astype(np.int64)


def _fill_parallel(n_heaps: int, lens: np.ndarray, body, threads: int | None):
    """Run ``body(h, out_slice)`` for every heap, writing into one flat array."""
    off = np.zeros(n_heaps + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    req = np.empty(int(off[-1]), dtype=np.int64)

    def work(lo_hi):
        for h in range(*lo_hi):
            body(h, req[off[h]:off[h + 1]])

    threads = threads or min(16, os.cpu_count() or 1)
    step = max(1, (n_heaps + 4 * threads - 1) // (4 * threads))
    chunks = [(a, min(a + step, n_heaps)) for a in range(0, n_heaps, step)]
    if threads <= 1 or len(chunks) <= 1:
        for c in chunks:
            work(c)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, chunks))
    return off, req


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def single_heap(seed: int = 1, n: int = 10_000, arena: int = 64 * KiB,
                align: int = 16, p_alloc: float = 0.6, lo: int = 16,
                hi: int = 4 * KiB, algo: int = FIRST_FIT) -> Batch:
    """One heap: 64 KiB arena, 16 B alignment, 10,000 steps, alloc w.p. 0.6
    with a size log-uniform on [16 B, 4 KiB], else free a uniform live block."""
    return uniform_batch(seed, 1, arena, align, n, p_alloc, lo, hi, algo,
                         name="single_heap_64KiB")


def uniform_batch(seed: int = 2, heaps: int = 4096, arena: int = 16 * MiB,
                  align: int = 64, n: int = 100_000, p_alloc: float = 0.55,
                  lo: int = 64, hi: int = 1 * MiB, algo: int = BEST_FIT,
                  name: str = "uniform_4096x16MiB", threads: int | None = None,
                  p_partial: float = 0.0) -> Batch:
    """Many identical heaps (default: 4,096 heaps of 16 MiB at 64 B alignment,
    100,000 requests each, sizes log-uniform on [64 B, 1 MiB], alloc w.p.
    0.55).  p_partial > 0 makes that fraction of the frees partial."""
    lens = np.full(heaps, n, dtype=np.int64)

    def body(h, out):
        rng = heap_rng(seed, h)
        sizes = log_uniform_int(rng, n, lo, hi)
        out[:] = _stream(rng, n, p_alloc, sizes, p_partial)

    off, req = _fill_parallel(heaps, lens, body, threads)
    return Batch(name, np.full(heaps, arena, np.int64),
                 np.full(heaps, align, np.int64), np.full(heaps, algo, np.int32),
                 off, req, dict(seed=seed, p_alloc=p_alloc, size_lo=lo,
                                size_hi=hi, steps=n, p_partial=p_partial))


def uneven_params(seed: int, heaps: int, arena_lo=1 * MiB, arena_hi=1 * GiB,
                  align=32, len_lo=1000, len_hi=1_000_000, alpha=1.5):
    """Per-heap arena (log-uniform, rounded down to the alignment), trace length
    (Pareto(alpha) scaled by len_lo, clipped) and algorithm (uniform over the
    four), drawn from a parameter stream separate from the request streams."""
    rng = np.random.Generator(np.random.PCG64(
        np.random.SeedSequence(entropy=seed, spawn_key=(1 << 30,))))
    a = log_uniform_int(rng, heaps, arena_lo, arena_hi)
    a = (a // align) * align
    u = rng.random(heaps)
    lens = np.floor(len_lo * (1.0 - u) ** (-1.0 / alpha))
    lens = np.clip(lens, len_lo, len_hi).astype(np.int64)
    algo = rng.integers(0, 4, heaps).astype(np.int32)
    return a.astype(np.int64), lens, algo


def uneven_batch(seed: int = 3, heaps: int = 16_384, p_alloc: float = 0.55,
                 align: int = 32, size_lo: int = 32, len_scale: float = 1.0,
                 threads: int | None = None, **kw) -> Batch:
    """Uneven batch: arena log-uniform [1 MiB, 1 GiB], lengths Pareto(1.5)
    clipped to [1k, 1M], algorithm uniform, sizes log-uniform [32 B, A/64].
    ``len_scale`` < 1 shortens every trace (for parity runs at reduced size)."""
    arena, lens, algo = uneven_params(seed, heaps, align=align, **kw)
    if len_scale != 1.0:
        lens = np.maximum(1, (lens * len_scale).astype(np.int64))

    def body(h, out):
        rng = heap_rng(seed, h)
        n = out.shape[0]
        sizes = log_uniform_int(rng, n, size_lo, arena[h] / 64)
        out[:] = _stream(rng, n, p_alloc, sizes)

    off, req = _fill_parallel(heaps, lens, body, threads)
    return Batch("uneven_16384", arena, np.full(heaps, align, np.int64), algo,
                 off, req, dict(seed=seed, p_alloc=p_alloc, len_scale=len_scale))


def geometric_class_sizes(rng: np.random.Generator, n: int, k_lo=12, k_hi=26,
                          gran=4096) -> np.ndarray:
    """Class k = k_lo + j with j ~ Geometric(1/2) truncated to [0, k_hi-k_lo]
    (renormalised); size uniform over the multiples of ``gran`` in
    (2^(k-1), 2^k]."""
    m = k_hi - k_lo + 1
    p = 0.5 ** (np.arange(m) + 1.0)
    cdf = np.cumsum(p / p.sum())
    cdf[-1] = 1.0
    j = np.searchsorted(cdf, rng.random(n), side="right")
    k = k_lo + j
    choices = np.maximum(1, (1 << np.maximum(k - 1, 0)) // gran)
    i = np.floor(rng.random(n) * choices).astype(np.int64)
    return (np.int64(1) << k) - gran * i


def large_seg_fit(seed: int = 5, n: int = 50_000_000, arena: int = 1 << 38,
                  align: int = 4096, p_alloc: float = 0.5) -> Batch:
    """One 256 GiB virtual heap at 4 KiB granularity, segregated fit, 50 M
    steps, alloc w.p. 0.5, sizes geometric over the 4 KiB..64 MiB classes."""
    rng = heap_rng(seed, 0)
    sizes = geometric_class_sizes(rng, n)
    req = _stream(rng, n, p_alloc, sizes)
    return Batch("large_seg_fit_256GiB", np.array([arena], np.int64),
                 np.array([align], np.int64), np.array([SEG_FIT], np.int32),
                 np.array([0, n], np.int64), req,
                 dict(seed=seed, p_alloc=p_alloc, steps=n))


def random_tiny(seed: int, n: int, granules: int, align: int = 16,
                p_alloc: float = 0.6, algo: int = FIRST_FIT,
                max_granules: int | None = None, p_partial: float = 0.0) -> Batch:
    """A small heap of ``granules`` * ``align`` bytes with sizes uniform on
    [0, max_granules * align] bytes (0 included, to exercise the minimum)."""
    rng = heap_rng(seed, 0)
    mg = max_granules or max(1, granules // 2)
    sizes = rng.integers(0, mg * align + 1, n, dtype=np.int64)
    req = _stream(rng, n, p_alloc, sizes, p_partial)
    return Batch("random_tiny", np.array([granules * align], np.int64),
                 np.array([align], np.int64), np.array([algo], np.int32),
                 np.array([0, n], np.int64), req, dict(seed=seed))


def paper_analog(seed: int = 6, n: int = 5_000, lo: int = 1 * KiB, hi: int = 16 * MiB,
                 p_alloc: float = 0.5, arena: int = 4 * GiB, align: int = 4 * KiB,
                 algo: int = SEG_FIT) -> Batch:
    """A stand-in for the paper's evaluation workload (random allocations and
    frees of blocks between 1 kB and 16 MB, several thousand times): n steps,
    allocate w.p. p_alloc with a size log-uniform on [lo, hi], else free a
    uniformly drawn live block; one heap (default: segregated fit over 4 GiB
    with 4 KiB granules, the setting the paper recommends for device
    memory)."""
    rng = heap_rng(seed, 0)
    sizes = log_uniform_int(rng, n, lo, hi)
    req = _stream(rng, n, p_alloc, sizes)
    return Batch("paper_analog", np.array([arena], np.int64), np.array([align], np.int64),
                 np.array([algo], np.int32), np.array([0, n], np.int64), req,
                 dict(seed=seed, p_alloc=p_alloc, size_lo=lo, size_hi=hi, steps=n))


def max_arena_batch(align: int = 64) -> Batch:
    """Hand-written traces on the largest arena a heap may have, 2^32 - 1
    granules: a block then ends at granule 2^32 - 1 and the whole free arena
    has size 2^32 - 1.  Trace 0 fills the arena with two blocks, frees and
    re-takes the one that ends there, then frees everything and asks for the
    whole arena; trace 1 does the same with sizes segregated fit can serve
    (the block ending at the arena end is exactly 2^31 granules).  Each trace
    runs once per algorithm (heap 4 * trace + algorithm)."""
    ag = (1 << 32) - 1
    g = align
    free = lambda r: -(r + 1)  # noqa: E731  (free with 32-bit draw r)
    last_of_two, first = 0xC0000000, 0
    t0 = [(1 << 31) * g, (ag - (1 << 31)) * g, free(last_of_two), 64, 128, free(first),
          free(0xFFFFFFFF), 4096, free(0x80000000), free(first), ag * g, free(first),
          ag * g, free(first)]
    t1 = [((1 << 31) - 1) * g, (1 << 31) * g, free(last_of_two), (1 << 31) * g,
          free(first), free(first), ag * g, 64, free(first), ((1 << 31) - 1) * g,
          (1 << 31) * g, free(last_of_two), free(first)]
    parts = []
    for t in (t0, t1):
        req = np.array(t, np.int64)
        for algo in ALGO_NAMES:
            parts.append(Batch("max_arena", np.array([ag * g], np.int64),
                               np.array([g], np.int64), np.array([algo], np.int32),
                               np.array([0, len(req)], np.int64), req))
    return concat(parts, "max_arena")


def concat(batches, name: str = "concat") -> Batch:
    """Concatenate batches heap-wise."""
    arena = np.concatenate([b.arena for b in batches])
    align = np.concatenate([b.align for b in batches])
    algo = np.concatenate([b.algo for b in batches])
    req = np.concatenate([b.req for b in batches])
    lens = np.concatenate([np.diff(b.req_off) for b in batches])
    off = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    return Batch(name, arena, align, algo, off, req)
