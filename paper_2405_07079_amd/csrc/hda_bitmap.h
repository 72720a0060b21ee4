// Bitmask allocator with a next-fit search (Sec. III-B), one wavefront per
// heap.  The heap's metadata is one flag per granule (set = free), 64 to a
// word, in device memory, plus the live table the replay driver frees from.
// An allocation of s granules takes the first s free granules in a row found
// scanning from the rover (the end of the last allocation), else from granule
// 0, and moves the rover past them; a free sets the flags back, so merging is
// implicit.
//
// The scan reads 64 words (4,096 granules) per step, one per lane.  For each
// lane the run of free granules that reaches the bottom of its word from
// below is found from the nearest lower lane whose word is not all free (a
// ballot, then a lane permute for that word's top run); a run that reaches
// s inside a word is found with s-1 shift-and steps.  The lowest start in the
// step is a wave-wide minimum.  Same rules as the other cores: values that
// feed a cross-lane operation are computed by all lanes with selects, never
// under a lane-dependent branch.
#pragma once
#include <stdint.h>

#include "hda_core.h"

namespace hda {

__device__ __forceinline__ uint32_t ctz64u(uint64_t m) {  // m != 0
  return (uint32_t)__builtin_ctzll(m);
}
__device__ __forceinline__ uint32_t clz64u(uint64_t m) {  // m != 0
  return (uint32_t)__builtin_clzll(m);
}
__device__ __forceinline__ uint32_t popc64(uint64_t m) {
  return (uint32_t)__builtin_popcountll(m);
}

// Inclusive prefix sum / maximum over the wave (row shifts inside 16-lane
// rows, then the row broadcasts), the pattern of wave_min.
__device__ __forceinline__ uint32_t wave_scan_add(uint32_t v) {
  v += row_shr<1>(0u, v);
  v += row_shr<2>(0u, v);
  v += row_shr<4>(0u, v);
  v += row_shr<8>(0u, v);
  v += row_bcast15(0u, v);
  v += row_bcast31(0u, v);
  return v;
}
__device__ __forceinline__ uint32_t wave_scan_max(uint32_t v) {
  v = max(v, row_shr<1>(0u, v));
  v = max(v, row_shr<2>(0u, v));
  v = max(v, row_shr<4>(0u, v));
  v = max(v, row_shr<8>(0u, v));
  v = max(v, row_bcast15(0u, v));
  v = max(v, row_bcast31(0u, v));
  return v;
}

struct BitHeap {
  HDA_GLOBAL uint64_t* bits;   // nw words: bit i of word w = granule 64 w + i free
  HDA_GLOBAL Ent* live;        // capL entries
  int64_t arena;
  uint32_t shift, ag, nw;
  uint32_t L, rover, capL;

  __device__ __forceinline__ BitHeap(uint64_t* b, Ent* lv, const HeapRegs& h, uint32_t cap_live)
      : bits((HDA_GLOBAL uint64_t*)b), live((HDA_GLOBAL Ent*)lv), arena(h.arena),
        shift(h.shift), ag(h.ag), nw((h.ag + 63u) >> 6), L(0), rover(0), capL(cap_live) {}

  // word wi, or 0 past the end (the load is clamped, not branched around)
  __device__ __forceinline__ uint64_t load(uint32_t wi) const {
    const uint64_t v = bits[wi < nw ? wi : nw - 1u];
    return wi < nw ? v : 0ull;
  }

  // Alg. 6: every granule free.
  __device__ void init() {
    for (uint32_t w0 = 0; w0 < nw; w0 += 64u) {
      const uint32_t wi = w0 + lane_id();
      const uint32_t rest = ag - 64u * (wi < nw ? wi : 0u);   // granules from this word on
      if (wi < nw) bits[wi] = rest >= 64u ? ~0ull : (1ull << rest) - 1ull;
    }
    L = 0;
    rover = 0;
  }

  // The lowest p >= lo with granules [p, p + s) all free, or kNone.  A run
  // is detected in the step holding its granule p + s - 1, so only starts
  // below `below_end` are wanted once steps begin at or past below_end + s.
  __device__ uint32_t find(uint32_t lo, uint32_t s, uint64_t below_end = 1ull << 40) const {
    const uint32_t lane = lane_id();
    uint64_t carry = 0;  // free granules in a row ending just below the step
    for (uint32_t w0 = lo >> 6; w0 < nw && 64ull * w0 < below_end + s; w0 += 64u) {
      const uint32_t wi = w0 + lane;
      const uint64_t below = wi == (lo >> 6) ? (1ull << (lo & 63u)) - 1ull : 0ull;
      const uint64_t w = load(wi) & ~below;
      const bool full = w == ~0ull;
      const uint32_t low1 = full ? 64u : ctz64u(~w);   // free run at the bottom
      const uint32_t top1 = full ? 64u : clz64u(~w);   // free run at the top
      // run reaching the bottom of this word: from the nearest lower lane
      // whose word is not all free, or from before the step
      const uint64_t lt = ballot(!full) & ((1ull << lane) - 1ull);
      const uint32_t ps = lt ? 63u - clz64u(lt) : 0u;
      const uint32_t tp = shfl(top1, ps);
      const uint64_t pre = lt ? (uint64_t)tp + 64ull * (lane - 1u - ps)
                              : carry + 64ull * lane;
      const uint64_t base = 64ull * wi;
      // a run that reaches s in this word, having started below it
      uint32_t cand = (pre < s && pre + low1 >= s) ? (uint32_t)(base - pre) : kNone;
      // a run of s inside this word
      if (s <= 64u) {
        uint64_t y = w;
        for (uint32_t k = 1; k < s;) {
          const uint32_t d = k < s - k ? k : s - k;
          y &= y >> d;
          k += d;
        }
        const uint32_t in = y ? (uint32_t)base + ctz64u(y) : kNone;
        cand = in < cand ? in : cand;
      }
      const uint32_t K = wave_min(cand);
      if (K != kNone) return K;
      const uint64_t topv = full ? pre + 64ull : (uint64_t)top1;
      carry = rdlane((uint32_t)topv, 63u);  // at most ag < 2^32
    }
    return kNone;
  }

  // Granules [p, p + s) become free (set) or used (cleared); one word per lane.
  __device__ void mark(uint32_t p, uint32_t s, bool set) {
    const uint32_t last = (p + s - 1u) >> 6;
    for (uint32_t w0 = p >> 6; w0 <= last; w0 += 64u) {
      const uint32_t wi = w0 + lane_id();
      if (wi <= last) {
        const uint64_t b0 = 64ull * wi;
        const uint32_t lo = (uint32_t)((uint64_t)p > b0 ? (uint64_t)p - b0 : 0ull);
        const uint64_t e = (uint64_t)p + s - b0;
        const uint32_t hi = (uint32_t)(e < 64ull ? e : 64ull);
        const uint64_t m = (hi == 64u ? ~0ull : (1ull << hi) - 1ull) & ~((1ull << lo) - 1ull);
        const uint64_t v = bits[wi];
        bits[wi] = set ? (v | m) : (v & ~m);
      }
    }
  }

  // Allocate sg granules (sg >= 1).  Returns the byte offset, -1 or kENoMeta.
  __device__ int64_t alloc(uint32_t sg, uint32_t) {
    if (sg > ag) return kFail;
    uint32_t p = find(rover, sg);
    // wrapping: starts at or past the rover were all tried
    if (p == kNone) p = find(0u, sg, rover);
    if (p == kNone) return kFail;
    if (L >= capL) return kENoMeta;
    mark(p, sg, false);
    live[L] = mk_ent(p, sg);  // every lane, same value
    ++L;
    rover = p + sg;
    return (int64_t)((uint64_t)p << shift);
  }

  // Replay free: the victim is live[(r * L) >> 32]; it keeps its first
  // floor(cut * size / 2^31) granules (partial deallocation); nothing live
  // -> -1.  Returns the byte offset of the freed part.
  __device__ int64_t free_draw(uint32_t r, uint32_t cut) {
    if (L == 0u) return kFail;
    const uint32_t idx = (uint32_t)(((uint64_t)r * (uint64_t)L) >> 32);
    const Ent e = live[idx];
    const uint32_t x = uniform(ent_a(e)), sz = uniform(ent_s(e));
    const uint32_t t = cut == 0u ? 0u : (uint32_t)(((uint64_t)cut * sz) >> 31);
    const Ent last = live[L - 1u];
    mark(x + t, sz - t, true);
    if (t != 0u) {
      live[idx] = mk_ent(x, t);
    } else {
      live[idx] = mk_ent(uniform(ent_a(last)), uniform(ent_s(last)));
      --L;
    }
    return (int64_t)((uint64_t)(x + t) << shift);
  }

  // Canonical state (format in hda.h): the free runs in address order, the
  // live table, the rover.
  __device__ int64_t dump(int64_t* out, int64_t cap) {
    const uint32_t lane = lane_id();
    uint32_t F = 0;
    for (uint32_t w0 = 0; w0 < nw; w0 += 64u) {
      const uint32_t wi = w0 + lane;
      const uint64_t w = load(wi);
      const uint64_t pw = wi > 0u ? load(wi - 1u) : 0ull;
      const uint64_t st = w & ~((w << 1) | (pw >> 63));  // first granule of a run
      F += rdlane(wave_scan_add(popc64(st)), 63u);
    }
    const int64_t need = 4 + 2 * (int64_t)F + 2 * (int64_t)L;
    if (out == nullptr || need > cap) return need;
    const uint32_t sh = shift;
    if (lane == 0) out[0] = F;
    int64_t* fo = out + 1;
    uint32_t done = 0, open = 0;  // runs written; start of the run open at the step's bottom
    for (uint32_t w0 = 0; w0 < nw; w0 += 64u) {
      const uint32_t wi = w0 + lane;
      const uint64_t w = load(wi);
      const uint64_t pw = wi > 0u ? load(wi - 1u) : 0ull;
      const uint64_t nx = load(wi + 1u);
      const uint64_t st = w & ~((w << 1) | (pw >> 63));        // run starts
      const uint64_t en = w & ~((w >> 1) | ((nx & 1ull) << 63)); // run ends (last granule)
      const uint32_t ne = popc64(en);
      const uint32_t incl = wave_scan_add(ne);
      // start of the run reaching this word from below: the last start in
      // the lower lanes of the step, or before the step (stored + 1, 0 = none)
      const uint32_t mine = st ? 64u * wi + 63u - clz64u(st) + 1u : 0u;
      const uint32_t upto = wave_scan_max(mine);
      const uint32_t prev = shfl(upto, (lane + 63u) & 63u);
      const uint32_t from = (lane != 0u && prev != 0u) ? prev - 1u : open;
      uint32_t k = done + incl - ne;
      for (uint64_t e = en; e != 0ull; e &= e - 1ull) {  // this lane's run ends
        const uint32_t b = ctz64u(e);
        const uint64_t sm = st & (b == 63u ? ~0ull : (2ull << b) - 1ull);
        const uint32_t a = sm ? 64u * wi + 63u - clz64u(sm) : from;
        const uint32_t end = 64u * wi + b + 1u;
        fo[2 * k] = (int64_t)((uint64_t)a << sh);
        fo[2 * k + 1] = (int64_t)((uint64_t)(end - a) << sh);
        ++k;
      }
      done += rdlane(incl, 63u);
      const uint32_t last = rdlane(upto, 63u);
      open = last != 0u ? last - 1u : open;
    }
    int64_t* lo = out + 1 + 2 * (int64_t)F;
    if (lane == 0) lo[0] = L;
    for (uint32_t base = 0; base < L; base += 64u) {
      const uint32_t i = base + lane;
      const Ent e = live[i < L ? i : 0u];
      if (i < L) {
        lo[1 + 2 * i] = (int64_t)((uint64_t)ent_a(e) << sh);
        lo[2 + 2 * i] = (int64_t)((uint64_t)ent_s(e) << sh);
      }
    }
    int64_t* tail = lo + 1 + 2 * (int64_t)L;
    if (lane == 0) {
      tail[0] = (int64_t)((uint64_t)rover << sh);
      tail[1] = 0;
    }
    return need;
  }
};

}  // namespace hda
