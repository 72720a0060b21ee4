// Device-side allocator core for gfx950: one 64-lane wavefront owns one heap.
//
// Metadata is out-of-band (Sec. III): nothing is stored in the managed arena,
// which is virtual.  Every heap keeps two tables of (granule address, granule
// size) pairs:
//
//  * the free table: one entry per free block, in no particular order.  The
//    whole wave searches it at once -- each lane tests the entries at its
//    lane index in 64-entry chunks, and a ballot or a DPP min-reduction picks
//    the winner -- so the sequential fits' "walk the address-ordered list"
//    (Sec. IV) becomes one associative pass:
//      first fit : min address among blocks with size >= s
//      next fit  : min address among fitting blocks whose end lies above the
//                  rover, else min address among all fitting blocks
//      best fit  : min (size, address) among fitting blocks
//    and neighbour lookup for coalescing (Alg. 2, Alg. 5) is a ballot for the
//    block ending at the freed address and the block starting at its end.
//    Insertion appends; removal moves the last entry into the hole.
//  * the live table: one entry per allocated block, in the replay driver's
//    order (append on allocation, last entry moved into the hole on free).
//
// Segregated fit (Alg. 4-5) keeps per-class LIFO lists.  Here a list is
// represented by push stamps: every push gives the block the next value of a
// per-heap clock, so the head of class k's list is the class-k block with the
// largest stamp and the list order head->tail is descending stamp order.
// Unlinking a block from the middle of a list leaves the others' relative
// order alone, exactly as pointer unlinking does.  Class occupancy counts live
// in one VGPR (lane k counts class k) and the availability bitmap is a ballot
// of the non-zero counts, so find-first-set on it (Sec. V-A) is one scalar
// instruction.
//
// Where the tables live: the first 64*RF free entries and 64*RL live entries
// are held in VGPRs (chunk r, lane l holds entry 64*r + l), so a scan is pure
// vector arithmetic and a single entry is read or written with readlane /
// writelane.  Entries past that ("cold") go to LDS and then to device memory;
// cold capacities are multiples of 64, so every 64-entry chunk lies wholly on
// one side and the side is chosen by a wave-uniform branch.
//
// The wavefront primitives (lane_id, ballot, rdlane, put_lane, uniform,
// row_shr, shfl, wave_sync) come from hda_wave.h, included before this
// header.  Values that feed a cross-lane operation are never produced under a
// lane-dependent branch (selects are used instead), so no lane can be sent
// round a loop on its own.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hda {

constexpr uint32_t kNone = 0xffffffffu;
constexpr int64_t kFail = -1, kEInval = -2, kEBadFree = -3, kENoMeta = -4,
                  kERange = -7;
enum : int { kFirstFit = 0, kNextFit = 1, kBestFit = 2, kSegFit = 3, kTlsf = 4, kBitmap = 5 };

// Wave-wide minimum of a u32; every lane must be active.  Row-local
// Hillis-Steele steps with DPP row shifts (identity shifted in) leave each
// row's minimum in its lane 15; two row broadcasts fold the four rows into
// lane 63.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
  const uint32_t I = 0xffffffffu;  // identity of unsigned min
  v = min(v, row_shr<1>(I, v));
  v = min(v, row_shr<2>(I, v));
  v = min(v, row_shr<4>(I, v));
  v = min(v, row_shr<8>(I, v));
  v = min(v, row_bcast15(I, v));
  v = min(v, row_bcast31(I, v));
  return rdlane(v, 63);
}

__device__ __forceinline__ uint32_t floor_log2_u32(uint32_t x) {  // x >= 1
  return 31u - (uint32_t)__builtin_clz(x);
}
__device__ __forceinline__ uint32_t ceil_log2_u32(uint32_t x) {   // x >= 1
  return x <= 1u ? 0u : 32u - (uint32_t)__builtin_clz(x - 1u);
}
__device__ __forceinline__ uint32_t ctz64(uint64_t m) {           // m != 0
  return (uint32_t)__builtin_ctzll(m);
}

// Two-level segregated fit (Sec. V-B): each power of two of the byte size is
// split into 2^kSli linear sub-classes.  A block of sg granules (sg >= 1, 2^shift
// bytes each) belongs to class index fl * 2^kSli + sl, fl = floor(log2 bytes);
// below 2^kSli bytes the sub-classes are finer than a byte and each holds
// one size.  In granules sl does not depend on the shift.
__host__ __device__ constexpr bool seg_like(int algo) { return algo == kSegFit || algo == kTlsf; }

constexpr uint32_t kSli = 5, kNsl = 1u << kSli;
constexpr uint32_t kTlsfClasses = 64u * kNsl;
__device__ __forceinline__ uint32_t tlsf_class(uint64_t sg, uint32_t shift) {
  const uint32_t lg = 63u - (uint32_t)__builtin_clzll(sg);
  const uint64_t sl = lg >= kSli ? (sg >> (lg - kSli)) - kNsl : (sg << (kSli - lg)) - kNsl;
  return (lg + shift) * kNsl + (uint32_t)sl;
}
// The class a request of sg granules is served from or above: its size
// rounded up to the next sub-class bound, so that every block of that class
// or a higher one fits (>= kTlsfClasses: nothing can).
__device__ __forceinline__ uint32_t tlsf_request_class(uint32_t sg, uint32_t shift) {
  const uint32_t lg = floor_log2_u32(sg);
  const uint64_t r = (uint64_t)sg + (lg >= kSli ? (1ull << (lg - kSli)) - 1ull : 0ull);
  return tlsf_class(r, shift);
}

// A table entry packs a block as (size << 32) | address, both in granules.
typedef uint64_t Ent;
__device__ __forceinline__ Ent mk_ent(uint32_t a, uint32_t s) { return ((uint64_t)s << 32) | a; }
__device__ __forceinline__ uint32_t ent_a(Ent e) { return (uint32_t)e; }
__device__ __forceinline__ uint32_t ent_s(Ent e) { return (uint32_t)(e >> 32); }

// Cold storage of a heap's tables: cold entry i of the free (live) table is
// at LDS index i while i < kf (kl), and at device index i - kf (i - kl) after.
struct Cold {
  HDA_LDS Ent* lf;           // LDS free entries
  HDA_LDS uint32_t* lst;     // LDS stamps
  HDA_LDS Ent* ll;           // LDS live entries
  HDA_GLOBAL Ent* gf;        // device free entries
  HDA_GLOBAL uint32_t* gst;  // device stamps
  HDA_GLOBAL Ent* gl;        // device live entries
  uint32_t kf, kl;           // LDS capacities (multiples of 64)
  uint32_t cf, cl;           // cold capacities (multiples of 64)
};

__device__ __forceinline__ Ent fget(const Cold& t, uint32_t i) {
  wave_sync();
  if (i < t.kf) return t.lf[i];
  return t.gf[i - t.kf];
}
__device__ __forceinline__ void fset(const Cold& t, uint32_t i, Ent e) {
  wave_sync();
  if (lane_id() == 0) {
    if (i < t.kf) t.lf[i] = e; else t.gf[i - t.kf] = e;
  }
}
__device__ __forceinline__ uint32_t sget(const Cold& t, uint32_t i) {
  wave_sync();
  if (i < t.kf) return t.lst[i];
  return t.gst[i - t.kf];
}
__device__ __forceinline__ void sset(const Cold& t, uint32_t i, uint32_t s) {
  wave_sync();
  if (lane_id() == 0) {
    if (i < t.kf) t.lst[i] = s; else t.gst[i - t.kf] = s;
  }
}
__device__ __forceinline__ Ent lget(const Cold& t, uint32_t i) {
  wave_sync();
  if (i < t.kl) return t.ll[i];
  return t.gl[i - t.kl];
}
__device__ __forceinline__ void lset(const Cold& t, uint32_t i, Ent e) {
  wave_sync();
  if (lane_id() == 0) {
    if (i < t.kl) t.ll[i] = e; else t.gl[i - t.kl] = e;
  }
}
// chunk loads: `base` is wave-uniform and a multiple of 64
__device__ __forceinline__ Ent fchunk(const Cold& t, uint32_t base) {
  wave_sync();
  if (base < t.kf) return t.lf[base + lane_id()];
  return t.gf[base - t.kf + lane_id()];
}
__device__ __forceinline__ uint32_t schunk(const Cold& t, uint32_t base) {
  wave_sync();
  if (base < t.kf) return t.lst[base + lane_id()];
  return t.gst[base - t.kf + lane_id()];
}
__device__ __forceinline__ Ent lchunk(const Cold& t, uint32_t base) {
  wave_sync();
  if (base < t.kl) return t.ll[base + lane_id()];
  return t.gl[base - t.kl + lane_id()];
}

// Wave-uniform heap registers.
struct HeapRegs {
  uint32_t F, L;      // free / live entries
  uint32_t ag;        // arena in granules
  uint32_t shift;     // log2(alignment)
  uint32_t rover;     // next fit: granule address where the next search resumes
  uint32_t clock;     // segregated fit: next push stamp
  int algo;
  int32_t status;     // first error seen on this heap
  int64_t arena;      // bytes
  uint32_t cnt;       // per lane: number of free blocks in class lane_id()
};

// One heap handled by one wave: RF free chunks and RL live chunks in VGPRs,
// the rest in `c`.  ALGO is fixed at compile time.
template <int ALGO, int RF, int RL>
struct WaveHeap {
  static constexpr uint32_t HF = 64u * RF, HL = 64u * RL;
  static constexpr int NF = RF > 0 ? RF : 1, NL = RL > 0 ? RL : 1;
  // segregated fit and TLSF: pushes are stamped; segregated fit alone keeps
  // per-class counts (TLSF's 2,048 classes are found by a reduction instead)
  static constexpr bool kSeg = ALGO == kSegFit || ALGO == kTlsf;
  static constexpr bool kCounts = ALGO == kSegFit;

  Cold c;
  HeapRegs h;
  uint32_t capF, capL;           // total table capacities
  uint32_t fa[NF], fs[NF], fst[NF];
  uint32_t la[NL], lz[NL];

  __device__ __forceinline__ WaveHeap(const Cold& cold, const HeapRegs& regs,
                                      uint32_t cap_free, uint32_t cap_live)
      : c(cold), h(regs), capF(cap_free), capL(cap_live) {}

  // ---- single entries (index wave-uniform) ----
  // Register chunks are addressed with selects on the uniform chunk index,
  // never with branches: a branch per chunk would make the compiler copy
  // every table register at each join.
  template <int R>
  __device__ __forceinline__ static uint32_t pick(const uint32_t (&v)[R], uint32_t r) {
    uint32_t x = opaque(v[0]);
#pragma unroll
    for (int k = 1; k < R; ++k) x = (r == (uint32_t)k) ? opaque(v[k]) : x;
    return x;
  }
  template <int R>
  __device__ __forceinline__ static void place(uint32_t (&v)[R], uint32_t r, uint32_t l,
                                               uint32_t x) {
    const bool me = lane_id() == l;
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = (me && r == (uint32_t)k) ? x : v[k];
  }

  __device__ __forceinline__ void fread(uint32_t i, uint32_t& a, uint32_t& s) {
    if (i < HF) {
      a = rdlane(pick(fa, i >> 6), i & 63u);
      s = rdlane(pick(fs, i >> 6), i & 63u);
    } else {
      const Ent e = fget(c, i - HF);
      a = ent_a(e); s = ent_s(e);
    }
  }
  __device__ __forceinline__ void fwrite(uint32_t i, uint32_t a, uint32_t s) {
    if (i < HF) {
      place(fa, i >> 6, i & 63u, a);
      place(fs, i >> 6, i & 63u, s);
    } else {
      fset(c, i - HF, mk_ent(a, s));
    }
  }
  __device__ __forceinline__ uint32_t stread(uint32_t i) {
    if (i < HF) return rdlane(pick(fst, i >> 6), i & 63u);
    return sget(c, i - HF);
  }
  __device__ __forceinline__ void stwrite(uint32_t i, uint32_t v) {
    if (i < HF) place(fst, i >> 6, i & 63u, v);
    else sset(c, i - HF, v);
  }
  __device__ __forceinline__ void lread(uint32_t i, uint32_t& a, uint32_t& s) {
    if (i < HL) {
      a = rdlane(pick(la, i >> 6), i & 63u);
      s = rdlane(pick(lz, i >> 6), i & 63u);
    } else {
      const Ent e = lget(c, i - HL);
      a = ent_a(e); s = ent_s(e);
    }
  }
  __device__ __forceinline__ void lwrite(uint32_t i, uint32_t a, uint32_t s) {
    if (i < HL) {
      place(la, i >> 6, i & 63u, a);
      place(lz, i >> 6, i & 63u, s);
    } else {
      lset(c, i - HL, mk_ent(a, s));
    }
  }

  // Free-table chunk at `base` (wave-uniform multiple of 64) for any base.
  __device__ __forceinline__ void fchunk_any(uint32_t base, uint32_t& a, uint32_t& s,
                                             uint32_t& st) {
    if (base < HF) {
      const uint32_t r = base >> 6;
      a = pick(fa, r); s = pick(fs, r); st = kSeg ? pick(fst, r) : 0u;
    } else {
      const Ent e = fchunk(c, base - HF);
      a = ent_a(e); s = ent_s(e);
      st = kSeg ? schunk(c, base - HF) : 0u;
    }
  }
  __device__ __forceinline__ void lchunk_any(uint32_t base, uint32_t& a, uint32_t& s) {
    if (base < HL) {
      const uint32_t r = base >> 6;
      a = pick(la, r); s = pick(lz, r);
    } else {
      const Ent e = lchunk(c, base - HL);
      a = ent_a(e); s = ent_s(e);
    }
  }

  // Visit every chunk of the free table: f(base, valid, a, s, stamp).  The
  // register chunks are all visited (entries past F are masked off), so the
  // register part needs no branch.
  template <typename Fn>
  __device__ __forceinline__ void scan_free(Fn&& f) {
#pragma unroll
    for (int k = 0; k < RF; ++k) {
      const uint32_t base = 64u * k;
      f(base, base + lane_id() < h.F, fa[k], fs[k], kSeg ? fst[k] : 0u);
    }
    for (uint32_t base = HF; base < h.F; base += 64u) {
      const Ent e = fchunk(c, base - HF);
      const uint32_t st = kSeg ? schunk(c, base - HF) : 0u;
      f(base, base + lane_id() < h.F, ent_a(e), ent_s(e), st);
    }
  }

  __device__ __forceinline__ uint32_t byte_class(uint32_t sg) const {
    return floor_log2_u32(sg) + h.shift;
  }
  // the list a free block of sg granules belongs to
  __device__ __forceinline__ uint32_t list_class(uint32_t sg) const {
    return ALGO == kTlsf ? tlsf_class(sg, h.shift) : byte_class(sg);
  }
  __device__ __forceinline__ void cnt_add(uint32_t cls, int d) {
    if (kCounts) h.cnt += (lane_id() == cls) ? (uint32_t)d : 0u;
  }
  __device__ __forceinline__ uint64_t class_bitmap() const { return ballot(h.cnt != 0u); }

  // Alg. 6: the free table starts as one block [0, A).
  __device__ __forceinline__ void init() {
    h.F = 1;
    h.L = 0;
    h.rover = 0;
    h.clock = 1;
    h.cnt = 0;
    fwrite(0, 0u, h.ag);
    if (kSeg) {
      stwrite(0, h.clock++);  // stamps start at 1: the key ~stamp never equals kNone
      cnt_add(byte_class(h.ag), 1);
    }
  }

  // Remove free entry j: the last entry moves into its place.
  __device__ __forceinline__ void fremove(uint32_t j) {
    const uint32_t last = h.F - 1u;
    if (j != last) {
      uint32_t a = 0, s = 0;
      fread(last, a, s);
      fwrite(j, a, s);
      if (kSeg) stwrite(j, stread(last));
    }
    h.F = last;
  }

  // Selection (Sec. II, Sec. IV, Sec. V-A).  Returns the chosen entry's index
  // or kNone; (ja, js) receive its address and size.  seg_lo is the chosen
  // class: in granule terms for segregated fit, the class index for TLSF.
  __device__ uint32_t select(uint32_t sg, uint32_t seg_lo, uint32_t& ja, uint32_t& js) {
    uint32_t k1 = kNone, k2 = kNone, bi = kNone, ba = 0, bs = 0;
    uint32_t w1 = kNone, wi = kNone, ws = 0;
    const uint32_t rover = h.rover;
    // lane-local updates are selects, not branches: their results feed the
    // wave-wide reductions below
    scan_free([&](uint32_t base, bool v, uint32_t a, uint32_t s, uint32_t st) {
      const uint32_t i = base + lane_id();
      if constexpr (ALGO == kFirstFit) {
        const bool take = v && s >= sg && a < k1;
        k1 = take ? a : k1; bi = take ? i : bi; bs = take ? s : bs;
      } else if constexpr (ALGO == kBestFit) {
        // keyed by the leftover s - sg (at most 2^32 - 2 since sg >= 1, so
        // it never equals kNone, as a whole-arena size of 2^32 - 1 would)
        const uint32_t d = s - sg;
        const bool take = v && s >= sg && (d < k1 || (d == k1 && a < k2));
        k1 = take ? d : k1; k2 = take ? a : k2; bi = take ? i : bi;
      } else if constexpr (ALGO == kNextFit) {
        const bool fit = v && s >= sg;
        const bool past = a + s > rover;
        const bool take = fit && past && a < k1;
        const bool wrap = fit && !past && a < w1;
        k1 = take ? a : k1; bi = take ? i : bi; bs = take ? s : bs;
        w1 = wrap ? a : w1; wi = wrap ? i : wi; ws = wrap ? s : ws;
      } else {  // segregated fit / TLSF: the class block pushed last
        // (lanes past the table may hold size 0, which has no class)
        const bool in = ALGO == kTlsf ? (v && s != 0u && list_class(s != 0u ? s : 1u) == seg_lo)
                                      : (s >> seg_lo) == 1u;
        const bool take = v && in && ~st < k1;
        k1 = take ? ~st : k1; bi = take ? i : bi; ba = take ? a : ba; bs = take ? s : bs;
      }
    });
    uint32_t K = wave_min(k1);
    if constexpr (ALGO == kNextFit) {
      if (K == kNone) {  // nothing fits past the rover: wrap around
        k1 = w1; bi = wi; bs = ws;
        K = wave_min(k1);
      }
    }
    if (K == kNone) return kNone;
    uint64_t m = ballot(k1 == K);
    if constexpr (ALGO == kBestFit) {
      // several lanes hold a block of the smallest size: lowest address wins
      if (__builtin_popcountll(m) > 1) {
        const uint32_t A2 = wave_min(k1 == K ? k2 : kNone);
        m = ballot(k1 == K && k2 == A2);
      }
      const uint32_t wl = ctz64(m);
      ja = rdlane(k2, wl);
      js = K + sg;
      return rdlane(bi, wl);
    } else {
      const uint32_t wl = ctz64(m);
      if constexpr (kSeg) ja = rdlane(ba, wl); else ja = K;
      js = rdlane(bs, wl);
      return rdlane(bi, wl);
    }
  }

  // Allocate sg granules (sg >= 1); k is the request's byte class for
  // segregated fit, its request class for TLSF.  Returns the byte offset,
  // -1, or kENoMeta (no change).
  __device__ int64_t alloc(uint32_t sg, uint32_t k) {
    uint32_t seg_lo = 0;
    if constexpr (ALGO == kSegFit) {
      if (k >= 64u) return kFail;
      const uint64_t m = class_bitmap() & (~0ull << k);
      if (m == 0ull) return kFail;
      seg_lo = ctz64(m) - h.shift;
    } else if constexpr (ALGO == kTlsf) {
      // the two-level bitmap lookup, as a reduction: the lowest class at or
      // above k that holds a free block
      if (k >= kTlsfClasses) return kFail;
      uint32_t m = kNone;
      scan_free([&](uint32_t, bool v, uint32_t, uint32_t s, uint32_t) {
        const uint32_t c = (v && s != 0u) ? list_class(s != 0u ? s : 1u) : kNone;
        m = (c >= k && c < m) ? c : m;
      });
      seg_lo = wave_min(m);
      if (seg_lo == kNone) return kFail;
    }
    uint32_t a = 0, bs = 0;
    const uint32_t j = select(sg, seg_lo, a, bs);
    if (j == kNone) return kFail;
    if (h.L >= capL) return kENoMeta;
    if (bs > sg) {  // Alg. 1 / Alg. 4: the block is cut from the low end
      fwrite(j, a + sg, bs - sg);
      if (kSeg) {
        stwrite(j, h.clock++);
        cnt_add(byte_class(bs), -1);
        cnt_add(byte_class(bs - sg), 1);
      }
    } else {
      fremove(j);
      if (kSeg) cnt_add(byte_class(bs), -1);
    }
    lwrite(h.L, a, sg);
    h.L++;
    if (ALGO == kNextFit) h.rover = a + sg;
    return (int64_t)((uint64_t)a << h.shift);
  }

  // Release block [x, x+sz) into the free table, merging with free
  // neighbours (Alg. 2 / Alg. 5).  Returns false (nothing changed) when the
  // table is full and a new entry would be needed.
  __device__ bool release(uint32_t x, uint32_t sz) {
    const uint32_t xe = x + sz;
    uint32_t jl = kNone, jr = kNone, sl = 0, sr = 0;
    scan_free([&](uint32_t base, bool v, uint32_t a, uint32_t s, uint32_t) {
      const uint64_t ml = ballot(v && a + s == x);
      const uint64_t mr = ballot(v && a == xe);
      if (ml) { const uint32_t w = ctz64(ml); jl = base + w; sl = rdlane(s, w); }
      if (mr) { const uint32_t w = ctz64(mr); jr = base + w; sr = rdlane(s, w); }
    });
    if (jl == kNone && jr == kNone) {
      if (h.F >= capF) return false;
      fwrite(h.F, x, sz);
      if (kSeg) { stwrite(h.F, h.clock++); cnt_add(byte_class(sz), 1); }
      h.F++;
    } else if (jr == kNone) {
      fwrite(jl, x - sl, sl + sz);
      if (kSeg) {
        stwrite(jl, h.clock++);
        cnt_add(byte_class(sl), -1);
        cnt_add(byte_class(sl + sz), 1);
      }
    } else if (jl == kNone) {
      fwrite(jr, x, sz + sr);
      if (kSeg) {
        stwrite(jr, h.clock++);
        cnt_add(byte_class(sr), -1);
        cnt_add(byte_class(sz + sr), 1);
      }
    } else {
      const uint32_t ms = sl + sz + sr;
      const uint32_t last = h.F - 1u;
      uint32_t keep;  // slot that ends up holding the merged block
      if (jr == last) {
        keep = jl;
      } else if (jl == last) {
        keep = jr;
      } else {
        keep = jl;
        uint32_t a = 0, s = 0;
        fread(last, a, s);
        fwrite(jr, a, s);
        if (kSeg) stwrite(jr, stread(last));
      }
      fwrite(keep, x - sl, ms);
      if (kSeg) {
        stwrite(keep, h.clock++);
        cnt_add(byte_class(sl), -1);
        cnt_add(byte_class(sr), -1);
        cnt_add(byte_class(ms), 1);
      }
      h.F = last;
    }
    return true;
  }

  // Free the live block at live-table index idx except its first t granules
  // (Alg. 2: t > 0 is a partial deallocation, the entry shrinks to t
  // granules; t = 0 frees the whole block and drops the entry).  Returns the
  // byte offset of the released part, or kENoMeta (state unchanged).
  __device__ int64_t free_index(uint32_t idx, uint32_t t = 0u) {
    uint32_t x = 0, sz = 0;
    lread(idx, x, sz);
    if (!release(x + t, sz - t)) return kENoMeta;
    if (t != 0u) {
      lwrite(idx, x, t);
      return (int64_t)((uint64_t)(x + t) << h.shift);
    }
    const uint32_t last = h.L - 1u;
    if (idx != last) {
      uint32_t a = 0, s = 0;
      lread(last, a, s);
      lwrite(idx, a, s);
    }
    h.L = last;
    return (int64_t)((uint64_t)x << h.shift);
  }

  // Replay-driver free: r is the 32-bit draw, the victim is
  // live[(r * L) >> 32]; the sequential fits keep its first
  // floor(cut * size / 2^31) granules (cut < 2^31); nothing live -> -1.
  __device__ __forceinline__ int64_t free_draw(uint32_t r, uint32_t cut = 0u) {
    if (h.L == 0u) return kFail;
    const uint32_t idx = (uint32_t)(((uint64_t)r * (uint64_t)h.L) >> 32);
    uint32_t t = 0u;
    if (!kSeg && cut != 0u) {
      uint32_t x = 0, sz = 0;
      lread(idx, x, sz);
      t = (uint32_t)(((uint64_t)cut * sz) >> 31);
    }
    return free_index(idx, t);
  }

  // Free by byte offset (the call-by-call interface): find the live entry.
  __device__ int64_t free_offset(int64_t off) {
    const uint64_t gm = (1ull << h.shift) - 1ull;
    if (off < 0 || off >= h.arena || ((uint64_t)off & gm)) return kEBadFree;
    const uint32_t x = (uint32_t)((uint64_t)off >> h.shift);
    uint32_t idx = kNone;
    for (uint32_t base = 0; base < h.L && idx == kNone; base += 64u) {
      uint32_t a = 0, s = 0;
      lchunk_any(base, a, s);
      const uint64_t m = ballot(base + lane_id() < h.L && a == x);
      if (m) idx = base + ctz64(m);
    }
    if (idx == kNone) return kEBadFree;
    const int64_t r = free_index(idx);
    return r < 0 ? r : 0;
  }

  // Partial free by byte offset (the call-by-call interface, Alg. 2): the
  // live block holding the offset keeps the part below it and the rest is
  // released; at a block's start this is a whole free.  Segregated fit frees
  // whole blocks only (Alg. 5): an interior offset is a bad free there.
  __device__ int64_t free_partial(int64_t off) {
    const uint64_t gm = (1ull << h.shift) - 1ull;
    if (off < 0 || off >= h.arena || ((uint64_t)off & gm)) return kEBadFree;
    const uint32_t x = (uint32_t)((uint64_t)off >> h.shift);
    uint32_t idx = kNone, t = 0u;
    for (uint32_t base = 0; base < h.L && idx == kNone; base += 64u) {
      uint32_t a = 0, s = 0;
      lchunk_any(base, a, s);
      // x - a < s (unsigned) holds exactly for a <= x < a + s
      const uint64_t m = ballot(base + lane_id() < h.L && x - a < s);
      if (m) {
        const uint32_t w = ctz64(m);
        idx = base + w;
        t = x - rdlane(a, w);
      }
    }
    if (idx == kNone || (kSeg && t != 0u)) return kEBadFree;
    const int64_t r = free_index(idx, t);
    return r < 0 ? r : 0;
  }

  // One allocation request of q >= 0 bytes (the call-by-call interface).
  __device__ int64_t alloc_bytes(int64_t q) {
    if (q > h.arena) return kFail;
    const uint64_t gm = (1ull << h.shift) - 1ull;
    uint32_t sg = (uint32_t)(((uint64_t)q + gm) >> h.shift);
    sg = sg == 0u ? 1u : sg;
    return alloc(sg, ALGO == kTlsf ? tlsf_request_class(sg, h.shift)
                                   : ceil_log2_u32(sg) + h.shift);
  }

  // Canonical state (format in hda.h), written by the whole wave.  The free
  // table is ranked by address and, for segregated fit, by descending stamp
  // within each class.  Returns the number of words (written only if <= cap).
  __device__ int64_t dump(int64_t* out, int64_t cap) {
    const uint32_t lane = lane_id();
    const int64_t lists = ALGO == kTlsf ? kTlsfClasses : 64;
    const int64_t need = 4 + 2 * (int64_t)h.F + 2 * (int64_t)h.L + (kSeg ? lists + (int64_t)h.F : 0);
    if (out == nullptr || need > cap) return need;
    const uint32_t sh = h.shift;
    if (lane == 0) out[0] = h.F;
    int64_t* fo = out + 1;
    for (uint32_t base = 0; base < h.F; base += 64u) {
      uint32_t a = 0, s = 0, st = 0;
      fchunk_any(base, a, s, st);
      const bool v = base + lane < h.F;
      uint32_t rank = 0;
      for (uint32_t j = 0; j < h.F; ++j) {
        uint32_t aj = 0, sj = 0;
        fread(j, aj, sj);
        rank += aj < a ? 1u : 0u;
      }
      if (v) {
        fo[2 * rank] = (int64_t)((uint64_t)a << sh);
        fo[2 * rank + 1] = (int64_t)((uint64_t)s << sh);
      }
    }
    int64_t* lo = out + 1 + 2 * (int64_t)h.F;
    if (lane == 0) lo[0] = h.L;
    for (uint32_t base = 0; base < h.L; base += 64u) {
      uint32_t a = 0, s = 0;
      lchunk_any(base, a, s);
      const uint32_t i = base + lane;
      if (i < h.L) {
        lo[1 + 2 * i] = (int64_t)((uint64_t)a << sh);
        lo[2 + 2 * i] = (int64_t)((uint64_t)s << sh);
      }
    }
    int64_t* tail = lo + 1 + 2 * (int64_t)h.L;
    uint64_t bm = class_bitmap();
    if constexpr (ALGO == kTlsf) {  // first level: the levels holding a free block
      bm = 0ull;
      for (uint32_t j = 0; j < h.F; ++j) {
        uint32_t aj = 0, sj = 0;
        fread(j, aj, sj);
        bm |= 1ull << (list_class(sj) / kNsl);
      }
    }
    if (lane == 0) {
      tail[0] = ALGO == kNextFit ? (int64_t)((uint64_t)h.rover << sh) : -1;
      tail[1] = kSeg ? (int64_t)bm : 0;
    }
    if constexpr (ALGO == kTlsf) {
      // list c starts at word c + (free blocks in lower classes); a block's
      // place in its list is the number of same-class blocks pushed later
      int64_t* ls = tail + 2;
      for (uint32_t c0 = 0; c0 < kTlsfClasses; c0 += 64u) {
        const uint32_t c = c0 + lane;
        uint32_t below = 0, n = 0;
        for (uint32_t j = 0; j < h.F; ++j) {
          uint32_t aj = 0, sj = 0;
          fread(j, aj, sj);
          const uint32_t cj = list_class(sj);
          below += cj < c ? 1u : 0u;
          n += cj == c ? 1u : 0u;
        }
        ls[c + below] = n;
      }
      for (uint32_t base = 0; base < h.F; base += 64u) {
        uint32_t a = 0, s = 0, st = 0;
        fchunk_any(base, a, s, st);
        const bool v = base + lane < h.F;
        const uint32_t cls = (v && s != 0u) ? list_class(s != 0u ? s : 1u) : kNone;
        uint32_t below = 0, rank = 0;
        for (uint32_t j = 0; j < h.F; ++j) {
          uint32_t aj = 0, sj = 0;
          fread(j, aj, sj);
          const uint32_t cj = list_class(sj), tj = stread(j);
          below += cj < cls ? 1u : 0u;
          rank += (cj == cls && tj > st) ? 1u : 0u;
        }
        if (v) ls[cls + below + 1u + rank] = (int64_t)((uint64_t)a << sh);
      }
    } else if constexpr (kSeg) {
      int64_t* ls = tail + 2;
      const uint32_t region = 64u + h.F;   // words of the class-list section
      // header position of class `lane`: sum over lower classes of (1 + count)
      uint32_t hdr = 0, acc = 0;
      for (uint32_t k = 0; k < 64u; ++k) {
        hdr = (lane == k) ? acc : hdr;
        acc += 1u + rdlane(h.cnt, k);
      }
      if (hdr < region) ls[hdr] = h.cnt;
      for (uint32_t base = 0; base < h.F; base += 64u) {
        uint32_t a = 0, s = 0, st = 0;
        fchunk_any(base, a, s, st);
        const bool v = base + lane < h.F;
        const uint32_t cls = v ? byte_class(s) : 0u;
        uint32_t rank = 0;
        for (uint32_t j = 0; j < h.F; ++j) {
          uint32_t aj = 0, sj = 0;
          fread(j, aj, sj);
          const uint32_t tj = stread(j);
          rank += (sj != 0u && byte_class(sj) == cls && tj > st) ? 1u : 0u;
        }
        const uint32_t hc = shfl(hdr, cls);
        if (v && hc + 1u + rank < region) ls[hc + 1u + rank] = (int64_t)((uint64_t)a << sh);
      }
    }
    return need;
  }
};

}  // namespace hda
