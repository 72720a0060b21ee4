// Lean replay core: one wavefront replays one heap with exactly two storage
// tiers.  Free-table entry i lives in lane i % 64 of 64-entry chunk i / 64;
// the first RF chunks are VGPRs and the rest LDS.  The wave's LDS region is
// one pool shared by both tables: free chunks from its start, live entries
// from its end, so a heap with many free blocks and one with many live
// blocks both fit.  Selection (Sec. II, Sec. IV, Sec. V-A) and the
// neighbour search of coalescing (Alg. 2, Alg. 5) are wave-wide scans over the
// chunks followed by one DPP reduction.
//
// Unused free slots hold address ~0 and size 0.  Such a slot never fits a
// request (every request is at least one granule) and never borders a block
// (no block starts at granule ~0; the one block that can end there, in an
// arena of 2^32 - 1 granules, is matched by its start instead), so every
// scan covers whole chunks with no bounds mask.
//
// When the tables would outgrow the pool before reaching the capacities the
// caller asked for, the request stops with kOverflow (changing nothing), the
// tables move into the general core's layout (hda_core.h, whose tables
// continue into device memory) and the heap goes on there.  Results are the
// same on both paths.
//
// Same rules as the general core: values that feed a cross-lane operation are
// never produced under a lane-dependent branch, and every LDS access is
// preceded by wave_sync().
#pragma once
#include <stdint.h>

#include "hda_core.h"

namespace hda {

constexpr int64_t kOverflow = -100;      // internal: the fast tiers are too small
// Segregated-fit key of a free block: the block's class in the top bits
// (6 for the 64 byte classes of segregated fit, 11 for the 2,048 classes of
// TLSF) and, below, the push stamp taken from the all-ones value (limit - 1 -
// stamp).  The smallest key at or above c << shift is then the head (the
// block pushed last) of the first non-empty class at or above c, so one
// wave-wide minimum does Alg. 4's class search (TLSF: the two-level bitmap
// lookup of Sec. V-B) and the list-head lookup together, and no per-class
// counts are kept on the request path.  Stamps start at 1, so a key never
// equals kNone, the key of an empty slot.
template <int ALGO>
struct SegKey {
  static constexpr uint32_t kShift = ALGO == kTlsf ? 21u : 26u;
  static constexpr uint32_t kLimit = 1u << kShift;   // stamps below this
  static constexpr uint32_t kMask = kLimit - 1u;
  static constexpr uint32_t kClasses = ALGO == kTlsf ? kTlsfClasses : 64u;
};

// Lane l of chunk r (both wave-uniform): every chunk's lane l is read and
// the right one chosen on the scalar unit, which keeps the read free of
// branches (a vector select chain here was turned into a branch ladder).
template <int R>
__device__ __forceinline__ uint32_t reg_lane(const uint32_t (&v)[R], uint32_t r, uint32_t l) {
  uint32_t x = rdlane(v[0], l);
#pragma unroll
  for (int k = 1; k < R; ++k) {
    const uint32_t y = rdlane(v[k], l);
    x = (r == (uint32_t)k) ? y : x;
  }
  return x;
}
// Lane l of chunk r becomes x; nothing changes when r >= R.
template <int R>
__device__ __forceinline__ void reg_place(uint32_t (&v)[R], uint32_t r, uint32_t l, uint32_t x) {
  const bool me = lane_id() == l;
#pragma unroll
  for (int k = 0; k < R; ++k) v[k] = (me && r == (uint32_t)k) ? x : v[k];
}

// The wave's LDS pool: `bytes` (a multiple of 16) from `base`.
struct LeanLds {
  HDA_LDS uint8_t* base;
  uint32_t bytes;
};

// A segregated-fit free entry in LDS: block and key in one 16-byte record
// (one 128-bit load); the other algorithms store just the 8-byte block.
struct __attribute__((aligned(16))) SegRec {
  uint32_t a, s, k, pad;
};

template <int ALGO, int RF>
struct LeanHeap {
  static constexpr bool kSeg = ALGO == kSegFit || ALGO == kTlsf;
  static constexpr uint32_t kKeyShift = SegKey<ALGO>::kShift;
  static constexpr uint32_t kStampLimit = SegKey<ALGO>::kLimit;
  static constexpr uint32_t kStampMask = SegKey<ALGO>::kMask;
  static constexpr uint32_t kClasses = SegKey<ALGO>::kClasses;
  static constexpr uint32_t HF = 64u * RF;
  static_assert(RF >= 1, "at least one register chunk");

  LeanLds m;
  uint32_t fa[RF], fs[RF], fk[RF];
  int64_t arena;
  uint32_t shift, ag;
  uint32_t F, L, rover, clock;
  uint32_t capF, capL;            // the caller's capacities (E_NOMETA past them)
  uint32_t live_room;             // live entries the pool holds beside the current free chunks

  __device__ __forceinline__ LeanHeap(const LeanLds& lds, const HeapRegs& h, uint32_t cap_free,
                                      uint32_t cap_live)
      : m(lds), arena(h.arena), shift(h.shift), ag(h.ag), capF(cap_free), capL(cap_live) {}

  // ---- the LDS pool ----
  static constexpr uint32_t kRec = kSeg ? 16u : 8u;  // bytes per free entry in LDS
  // Pool bytes the tables take with f free and l live entries: the free
  // entries past the register chunks in whole 64-entry chunks (scans read
  // whole chunks), then the live entries.
  __device__ __forceinline__ uint32_t need_bytes(uint32_t f, uint32_t l) const {
    const uint32_t cold = f > HF ? f - HF : 0u;
    return ((cold + 63u) & ~63u) * kRec + l * 8u;
  }
  // Recompute live_room after F changed.
  __device__ __forceinline__ void set_room() {
    const uint32_t cold = F > HF ? F - HF : 0u;
    const uint32_t used = ((cold + 63u) & ~63u) * kRec;
    live_room = used <= m.bytes ? (m.bytes - used) >> 3 : 0u;
  }
  // LDS free entry i (free-table index HF + i).
  __device__ __forceinline__ void cold_get(uint32_t i, uint32_t& a, uint32_t& s,
                                           uint32_t& k) const {
    if constexpr (kSeg) {
      // the whole record in one 16-byte load (a 4-byte load of the key
      // alone, 16 bytes apart per lane, meets bank conflicts)
      typedef uint32_t rec4 __attribute__((vector_size(16)));
      const rec4 v = *((const HDA_LDS rec4*)m.base + i);
      a = v[0]; s = v[1]; k = v[2];
    } else {
      const Ent e = ((HDA_LDS Ent*)m.base)[i];
      a = ent_a(e); s = ent_s(e); k = 0u;
    }
  }
  __device__ __forceinline__ void cold_put(uint32_t i, uint32_t a, uint32_t s, uint32_t k) const {
    if constexpr (kSeg) {
      HDA_LDS SegRec* r = (HDA_LDS SegRec*)m.base + i;
      r->a = a; r->s = s; r->k = k; r->pad = 0u;
    } else {
      ((HDA_LDS Ent*)m.base)[i] = mk_ent(a, s);
    }
  }
  // Live entry i, counted from the end of the pool.
  __device__ __forceinline__ HDA_LDS Ent* live_ptr(uint32_t i) const {
    return (HDA_LDS Ent*)(m.base + m.bytes) - (i + 1u);
  }

  // the list a free block of sg granules belongs to
  __device__ __forceinline__ uint32_t list_class(uint32_t sg) const {
    return ALGO == kTlsf ? tlsf_class(sg, shift) : floor_log2_u32(sg) + shift;
  }
  __device__ __forceinline__ uint32_t seg_key(uint32_t sg) {
    return (list_class(sg) << kKeyShift) | (clock++ ^ kStampMask);
  }
  // Segregated fit, lane k: the number of free blocks of byte class k (for
  // the canonical state and the hand-over to the general core; not kept per
  // request).
  __device__ uint32_t class_counts() {
    uint32_t n = 0;
    for (uint32_t j = 0; j < F; ++j) {
      uint32_t a, s, k;
      read(j, a, s, k);
      n += lane_id() == (k >> kKeyShift) ? 1u : 0u;
    }
    return n;
  }

  // ---- free-table entries by wave-uniform index ----
  __device__ __forceinline__ uint32_t size_at(uint32_t j) {
    if (j < HF) return reg_lane(fs, j >> 6, j & 63u);
    wave_sync();
    uint32_t a, s, k;
    cold_get(j - HF, a, s, k);
    return uniform(s);
  }
  __device__ __forceinline__ void read(uint32_t j, uint32_t& a, uint32_t& s, uint32_t& k) {
    if (j < HF) {
      const uint32_t r = j >> 6, l = j & 63u;
      a = reg_lane(fa, r, l);
      s = reg_lane(fs, r, l);
      k = kSeg ? reg_lane(fk, r, l) : 0u;
    } else {
      wave_sync();
      uint32_t ea, es, ek;
      cold_get(j - HF, ea, es, ek);
      a = uniform(ea);
      s = uniform(es);
      k = kSeg ? uniform(ek) : 0u;
    }
  }
  // The block (address, size) of free entry j.
  __device__ __forceinline__ void read_block(uint32_t j, uint32_t& a, uint32_t& s) {
    if (j < HF) {
      const uint32_t r = j >> 6, l = j & 63u;
      a = reg_lane(fa, r, l);
      s = reg_lane(fs, r, l);
    } else {
      wave_sync();
      uint32_t ea, es, ek;
      cold_get(j - HF, ea, es, ek);
      a = uniform(ea);
      s = uniform(es);
    }
  }
  // The register chunks take a select each (none matches a cold index), so
  // the tables are never merged across a branch.  An LDS entry is stored by
  // every lane with the same value: a store guarded by a lane test would be
  // merged by the optimiser with the uniform test around it into one
  // divergent branch, which turns the heap's counters into per-lane values.
  __device__ __forceinline__ void write(uint32_t j, uint32_t a, uint32_t s, uint32_t k) {
    const uint32_t r = j >> 6, l = j & 63u;
    reg_place(fa, r, l, a);
    reg_place(fs, r, l, s);
    if (kSeg) reg_place(fk, r, l, k);
    if (j >= HF) {
      wave_sync();
      cold_put(j - HF, a, s, k);
    }
  }
  __device__ __forceinline__ void clear(uint32_t j) { write(j, kNone, 0u, kNone); }

  // ---- live table ----
  __device__ __forceinline__ void live_read(uint32_t i, uint32_t& a, uint32_t& s) {
    wave_sync();
    const Ent e = *live_ptr(i);
    a = uniform(ent_a(e));
    s = uniform(ent_s(e));
  }
  __device__ __forceinline__ void live_write(uint32_t i, uint32_t a, uint32_t s) {
    wave_sync();
    *live_ptr(i) = mk_ent(a, s);  // every lane, same value (see write())
  }

  // Visit every chunk holding entries: f(chunk, a, s, key).  LDS chunks are
  // loaded four at a time before any is used, so their latencies overlap.
  template <typename Fn>
  __device__ __forceinline__ void scan(Fn&& f) {
#pragma unroll
    for (int k = 0; k < RF; ++k) f((uint32_t)k, fa[k], fs[k], kSeg ? fk[k] : 0u);
    uint32_t c = RF;
    for (; 64u * (c + 3u) < F; c += 4u) {
      const uint32_t i = 64u * (c - RF) + lane_id();
      wave_sync();
      uint32_t ea[4], es[4], ek[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) cold_get(i + 64u * u, ea[u], es[u], ek[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) f(c + u, ea[u], es[u], ek[u]);
    }
    for (; 64u * c < F; ++c) {
      const uint32_t i = 64u * (c - RF) + lane_id();
      wave_sync();
      uint32_t ea, es, ek;
      cold_get(i, ea, es, ek);
      f(c, ea, es, ek);
    }
  }

  // Alg. 6: one free block [0, A).
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int k = 0; k < RF; ++k) { fa[k] = kNone; fs[k] = 0u; fk[k] = kNone; }
    F = 1; L = 0; rover = 0; clock = 1;
    set_room();
    write(0, 0u, ag, kSeg ? seg_key(ag) : 0u);
  }

  // Remove free entry j: the last entry moves into its place and the last
  // slot is cleared.
  template <bool CHK = true>
  __device__ __forceinline__ void remove(uint32_t j) {
    // no branch on j == last: moving the last entry onto itself is harmless,
    // and a branch here made the compiler copy the register chunks
    const uint32_t last = F - 1u;
    uint32_t a, s, k;
    read(last, a, s, k);
    write(j, a, s, k);
    clear(last);
    F = last;
    if (CHK) set_room();
  }

  // Selection.  On success j is the chosen entry and (a, s) its block.
  __device__ __forceinline__ bool select(uint32_t sg, uint32_t kreq, uint32_t& j, uint32_t& a,
                                         uint32_t& s) {
    if constexpr (ALGO == kFirstFit || ALGO == kNextFit) {
      // first fit: lowest address among blocks that fit.  Next fit: blocks
      // are taken in cyclic order starting at the first whose end is past the
      // rover; since free blocks do not overlap, that order is the order of
      // end - rover - 1 taken mod 2^32.  The block ending exactly at the rover
      // (last in that order) has key ~0, which the scan cannot tell from
      // "none", so it is looked for separately when nothing else fits.
      const uint32_t nr = ~rover;
      uint32_t best = kNone, bc = 0, bsz = 0;  // bsz: the candidate's size
      scan([&](uint32_t c, uint32_t ea, uint32_t es, uint32_t) {
        const uint32_t t = es >= sg ? (ALGO == kFirstFit ? ea : ea + es + nr) : kNone;
        const bool lt = t < best;
        best = lt ? t : best;
        bc = lt ? c : bc;
        bsz = lt ? es : bsz;
      });
      const uint32_t K = wave_min(best);
      uint64_t mk;
      uint32_t end;  // next fit: end of the chosen block
      if (K != kNone) {
        mk = ballot(best == K);
        end = K - nr;
      } else {
        if (ALGO == kFirstFit) return false;
        uint64_t any = 0ull;
        scan([&](uint32_t c, uint32_t ea, uint32_t es, uint32_t) {
          const bool hit = es >= sg && ea + es == rover;
          any |= ballot(hit);
          bc = hit ? c : bc;
          bsz = hit ? es : bsz;
        });
        if (any == 0ull) return false;
        mk = any;
        end = rover;
      }
      const uint32_t l = ctz64(mk);
      j = 64u * rdlane(bc, l) + l;
      s = rdlane(bsz, l);
      a = ALGO == kFirstFit ? K : end - s;
      return true;
    } else if constexpr (ALGO == kBestFit) {
      // smallest size, then lowest address: (leftover, address) compared as
      // one 64-bit value, one vector compare per chunk.  The leftover is
      // es - sg mod 2^32: a block that fits leaves at most ~sg, one that
      // does not (empty slots included, size 0) wraps to more, so no test
      // of the size is needed per entry.
      uint64_t best = ~0ull;
      uint32_t bc = 0;
      scan([&](uint32_t c, uint32_t ea, uint32_t es, uint32_t) {
        const uint64_t key = ((uint64_t)(es - sg) << 32) | ea;
        const bool take = key < best;
        best = take ? key : best;
        bc = take ? c : bc;
      });
      const uint32_t bs = (uint32_t)(best >> 32), ba = (uint32_t)best;
      const uint32_t K = wave_min(bs);
      if (K > ~sg) return false;
      uint64_t mk = ballot(bs == K);
      if (__builtin_popcountll(mk) > 1) {
        const uint32_t A2 = wave_min(bs == K ? ba : kNone);
        mk = ballot(bs == K && ba == A2);
      }
      const uint32_t l = ctz64(mk);
      j = 64u * rdlane(bc, l) + l;
      a = rdlane(ba, l);
      s = K + sg;
      return true;
    } else {
      // segregated fit: the first non-empty class at or above the request's,
      // and in it the block pushed last (Alg. 4): the smallest key at or
      // above the request's class
      if (kreq >= kClasses) return false;
      const uint32_t lo = kreq << kKeyShift;
      // Keys are compared as (key - lo) mod 2^32: keys below lo wrap past
      // every key at or above it and past the empty slots' key ~0 (which
      // maps to ~lo), so the smallest such value is the smallest key at or
      // above lo whenever it is below ~lo.  Only the chunk is carried; the
      // block is read from the chosen slot afterwards.
      uint32_t best = kNone, bc = 0;
      scan([&](uint32_t ch, uint32_t, uint32_t, uint32_t ek) {
        const uint32_t t = ek - lo;
        const bool lt = t < best;
        best = lt ? t : best;
        bc = lt ? ch : bc;
      });
      const uint32_t K = wave_min(best);
      if (K >= ~lo) return false;
      const uint32_t l = ctz64(ballot(best == K));
      j = 64u * rdlane(bc, l) + l;
      read_block(j, a, s);
      return true;
    }
  }

  // Allocate sg granules; kreq is the request's byte class (segregated fit).
  // Returns the byte offset, -1, kENoMeta or kOverflow.
  // CHK = false: the caller has established that no request of the current
  // block can outgrow the tiers or reach the capacities (block_safe), so
  // those checks and the upkeep of live_room are left out; live_room is
  // refreshed after the block.
  template <bool CHK = true>
  __device__ __forceinline__ int64_t alloc(uint32_t sg, uint32_t kreq) {
    uint32_t j = 0, a = 0, s = 0;
    if (!select(sg, kreq, j, a, s)) return kFail;
    if (CHK && L >= capL) return kENoMeta;
    if (CHK && L >= live_room) return kOverflow;
    if (s > sg) {  // Alg. 1 / Alg. 4: the block is cut from the low end
      if (CHK && kSeg && clock >= kStampLimit) return kOverflow;
      write(j, a + sg, s - sg, kSeg ? seg_key(s - sg) : 0u);
    } else {
      remove<CHK>(j);
    }
    live_write(L, a, sg);
    ++L;
    if (ALGO == kNextFit) rover = a + sg;
    return (int64_t)((uint64_t)a << shift);
  }

  // Free live entry idx except its first floor(cut * size / 2^31) granules
  // (partial deallocation, sequential fits only; cut < 2^31): coalesce the
  // released part with free neighbours (Alg. 2 / Alg. 5), then shrink the
  // entry or, for a whole free, drop it from the live table (the last one
  // moves into its place).  Returns the byte offset of the released part,
  // kENoMeta or kOverflow.
  template <bool CHK = true>
  __device__ __forceinline__ int64_t free_index(uint32_t idx, uint32_t cut) {
    if (CHK && kSeg && clock >= kStampLimit) return kOverflow;
    // The victim and the last live entry (which takes the victim's slot at
    // the end) are read together, so the second load's latency hides behind
    // the first; nothing below writes the live table before that move.
    const uint32_t lastL = L - 1u;
    uint32_t bx, bsz, ta, ts;
    live_read(idx, bx, bsz);
    live_read(lastL, ta, ts);
    const uint32_t t = (kSeg || cut == 0u) ? 0u : (uint32_t)(((uint64_t)cut * bsz) >> 31);
    const uint32_t x = bx + t, sz = bsz - t;  // the part released
    // A block ending at granule ~0 (an arena of 2^32 - 1 granules) has no
    // right neighbour; its own start, which no free block has, stands in for
    // its end so that empty slots (address ~0) do not match.
    const uint32_t xe = x + sz == kNone ? x : x + sz;
    // chunk + 1 of this lane's left / right neighbour (0: none); there is at
    // most one of each, so two ballots after the scan find them
    uint32_t cl = 0, cr = 0;
    scan([&](uint32_t c, uint32_t ea, uint32_t es, uint32_t) {
      cl = ea + es == x ? c + 1u : cl;
      cr = ea == xe ? c + 1u : cr;
    });
    const uint64_t ML = ballot(cl != 0u), MR = ballot(cr != 0u);
    if ((ML | MR) == 0ull) {
      if (CHK && F >= capF) return kENoMeta;
      // (the freed block still counts as live here: the check is on the safe side)
      if (CHK && need_bytes(F + 1u, L) > m.bytes) return kOverflow;
      if (F >= HF && ((F - HF) & 63u) == 0u) {  // a new LDS chunk: its slots start empty
        wave_sync();
        cold_put(F - HF + lane_id(), kNone, 0u, kNone);
      }
      write(F, x, sz, kSeg ? seg_key(sz) : 0u);
      ++F;
      if (CHK) set_room();
    } else if (MR == 0ull) {
      const uint32_t l = ctz64(ML), jl = 64u * (rdlane(cl, l) - 1u) + l;
      const uint32_t sl = size_at(jl);
      write(jl, x - sl, sl + sz, kSeg ? seg_key(sl + sz) : 0u);
    } else if (ML == 0ull) {
      const uint32_t l = ctz64(MR), jr = 64u * (rdlane(cr, l) - 1u) + l;
      const uint32_t sr = size_at(jr);
      write(jr, x, sz + sr, kSeg ? seg_key(sz + sr) : 0u);
    } else {
      const uint32_t ll = ctz64(ML), jl = 64u * (rdlane(cl, ll) - 1u) + ll;
      const uint32_t lr = ctz64(MR), jr = 64u * (rdlane(cr, lr) - 1u) + lr;
      const uint32_t sl = size_at(jl), sr = size_at(jr), ms = sl + sz + sr;
      const uint32_t last = F - 1u;
      uint32_t keep = 0;  // slot that ends up holding the merged block
      if (jr == last) {
        keep = jl;
      } else if (jl == last) {
        keep = jr;
      } else {
        keep = jl;
        uint32_t a, s, k;
        read(last, a, s, k);
        write(jr, a, s, k);
      }
      write(keep, x - sl, ms, kSeg ? seg_key(ms) : 0u);
      clear(last);
      F = last;
      if (CHK) set_room();
    }
    if (t != 0u) {
      live_write(idx, bx, t);
    } else {
      live_write(idx, ta, ts);  // idx == lastL rewrites the entry about to be dropped
      L = lastL;
    }
    return (int64_t)((uint64_t)x << shift);
  }

  // Replay free: r is the 32-bit draw, the victim is live[(r * L) >> 32];
  // cut as in free_index; nothing live -> -1.
  template <bool CHK = true>
  __device__ __forceinline__ int64_t free_draw(uint32_t r, uint32_t cut) {
    if (CHK && L == 0u) return kFail;
    return free_index<CHK>((uint32_t)(((uint64_t)r * (uint64_t)L) >> 32), cut);
  }

  // Whether the next n (<= 64) requests can skip the overflow and capacity
  // checks: each adds at most one live entry and one free entry, n free
  // entries open at most one new LDS chunk (64 entries of kRec bytes, the
  // room of 8 kRec live entries), and each takes at most one push stamp;
  // with n live blocks to start from, no free finds the live table empty.
  __device__ __forceinline__ bool block_safe(uint32_t n) const {
    return L + n + 8u * kRec <= live_room && L + n <= capL && F + n <= capF && L >= n &&
           (!kSeg || clock + n < kStampLimit);
  }

  // Hand this heap over to the general core (hda_core.h) on tiers `c` with
  // no LDS part: every free entry i goes to device slot i with its push stamp
  // beside it, every live entry i to device slot i.
  __device__ void migrate(const Cold& c, HeapRegs& h) {
    const uint32_t lane = lane_id();
    const uint32_t counts = ALGO == kSegFit ? class_counts() : 0u;
    for (uint32_t ch = RF; 64u * ch < F; ++ch) {
      const uint32_t gi = 64u * ch + lane;
      wave_sync();
      uint32_t a, s, k;
      cold_get(64u * (ch - RF) + lane, a, s, k);
      if (gi < F) {
        c.gf[gi] = mk_ent(a, s);
        if (kSeg) c.gst[gi] = (k & kStampMask) ^ kStampMask;
      }
    }
#pragma unroll
    for (int k = 0; k < RF; ++k) {
      const uint32_t gi = 64u * (uint32_t)k + lane;
      if (gi < F) {
        c.gf[gi] = mk_ent(fa[k], fs[k]);
        if (kSeg) c.gst[gi] = (fk[k] & kStampMask) ^ kStampMask;
      }
    }
    for (uint32_t base = 0; base < L; base += 64u) {
      const uint32_t i = base + lane;
      wave_sync();
      const Ent e = *live_ptr(i < L ? i : 0u);
      if (i < L) c.gl[i] = e;
    }
    wave_sync();
    h.F = F;
    h.L = L;
    h.rover = rover;
    h.clock = clock;
    h.cnt = counts;
  }

  // Canonical state, same format as the general core (hda.h).
  __device__ int64_t dump(int64_t* out, int64_t cap) {
    const uint32_t lane = lane_id();
    const int64_t need = 4 + 2 * (int64_t)F + 2 * (int64_t)L + (kSeg ? kClasses + (int64_t)F : 0);
    if (out == nullptr || need > cap) return need;
    const uint32_t sh = shift;
    if (lane == 0) out[0] = F;
    int64_t* fo = out + 1;
    // free blocks ranked by address
    scan([&](uint32_t c, uint32_t a, uint32_t s, uint32_t) {
      const bool v = 64u * c + lane < F;
      uint32_t rank = 0;
      for (uint32_t j = 0; j < F; ++j) {
        uint32_t aj, sj, kj;
        read(j, aj, sj, kj);
        rank += aj < a ? 1u : 0u;
      }
      if (v) {
        fo[2 * rank] = (int64_t)((uint64_t)a << sh);
        fo[2 * rank + 1] = (int64_t)((uint64_t)s << sh);
      }
    });
    int64_t* lo = out + 1 + 2 * (int64_t)F;
    if (lane == 0) lo[0] = L;
    for (uint32_t base = 0; base < L; base += 64u) {
      const uint32_t i = base + lane;
      wave_sync();
      const Ent e = *live_ptr(i < L ? i : 0u);
      if (i < L) {
        lo[1 + 2 * i] = (int64_t)((uint64_t)ent_a(e) << sh);
        lo[2 + 2 * i] = (int64_t)((uint64_t)ent_s(e) << sh);
      }
    }
    int64_t* tail = lo + 1 + 2 * (int64_t)L;
    const uint32_t cnt = ALGO == kSegFit ? class_counts() : 0u;
    uint64_t bm = ballot(cnt != 0u);
    if constexpr (ALGO == kTlsf) {  // first level: the levels holding a free block
      bm = 0ull;
      for (uint32_t j = 0; j < F; ++j) {
        uint32_t aj, sj, kj;
        read(j, aj, sj, kj);
        bm |= 1ull << ((kj >> kKeyShift) / kNsl);
      }
    }
    if (lane == 0) {
      tail[0] = ALGO == kNextFit ? (int64_t)((uint64_t)rover << sh) : -1;
      tail[1] = kSeg ? (int64_t)bm : 0;
    }
    if constexpr (ALGO == kTlsf) {
      // list c starts at word c + (free blocks in lower classes); a block's
      // place in its list is the number of same-class blocks pushed later
      // (smaller keys)
      int64_t* ls = tail + 2;
      for (uint32_t c0 = 0; c0 < kClasses; c0 += 64u) {
        const uint32_t cl = c0 + lane;
        uint32_t below = 0, n = 0;
        for (uint32_t j = 0; j < F; ++j) {
          uint32_t aj, sj, kj;
          read(j, aj, sj, kj);
          below += (kj >> kKeyShift) < cl ? 1u : 0u;
          n += (kj >> kKeyShift) == cl ? 1u : 0u;
        }
        ls[cl + below] = n;
      }
      scan([&](uint32_t c, uint32_t a, uint32_t, uint32_t key) {
        const bool v = 64u * c + lane < F;
        const uint32_t cls = key >> kKeyShift;
        uint32_t below = 0, rank = 0;
        for (uint32_t j = 0; j < F; ++j) {
          uint32_t aj, sj, kj;
          read(j, aj, sj, kj);
          below += (kj >> kKeyShift) < cls ? 1u : 0u;
          rank += ((kj >> kKeyShift) == cls && kj < key) ? 1u : 0u;
        }
        if (v) ls[cls + below + 1u + rank] = (int64_t)((uint64_t)a << sh);
      });
    } else if constexpr (kSeg) {
      int64_t* ls = tail + 2;
      const uint32_t region = 64u + F;  // words of the class-list section
      // header position of class `lane`: sum over lower classes of (1 + count)
      uint32_t hdr = 0, acc = 0;
      for (uint32_t k = 0; k < 64u; ++k) {
        hdr = (lane == k) ? acc : hdr;
        acc += 1u + rdlane(cnt, k);
      }
      if (hdr < region) ls[hdr] = cnt;
      // within a class, blocks from the last pushed (smallest key) on
      scan([&](uint32_t c, uint32_t a, uint32_t, uint32_t key) {
        const bool v = 64u * c + lane < F;
        const uint32_t cls = v ? key >> kKeyShift : 0u;
        uint32_t rank = 0;
        for (uint32_t j = 0; j < F; ++j) {
          uint32_t aj, sj, kj;
          read(j, aj, sj, kj);
          rank += ((kj >> kKeyShift) == cls && kj < key) ? 1u : 0u;
        }
        const uint32_t hc = shfl(hdr, cls);
        if (v && hc + 1u + rank < region) ls[hc + 1u + rank] = (int64_t)((uint64_t)a << sh);
      });
    }
    return need;
  }
};

}  // namespace hda
