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
// The first kf free entries and kl live entries of a heap sit in LDS; later
// entries spill to a per-wave region of device memory (kf, kl are multiples of
// 64, so every 64-entry chunk lies wholly on one side and the side is chosen by
// a wave-uniform branch).
//
// The wavefront primitives (lane_id, ballot, rdlane, uniform, row_shr, shfl,
// wave_sync) come from hda_wave.h, included before this header.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hda {

constexpr uint32_t kNone = 0xffffffffu;
constexpr int64_t kFail = -1, kEInval = -2, kEBadFree = -3, kENoMeta = -4,
                  kERange = -7;
enum : int { kFirstFit = 0, kNextFit = 1, kBestFit = 2, kSegFit = 3 };

// Wave-wide minimum of a u32; every lane must be active.  Row-local
// Hillis-Steele steps with DPP row shifts (identity shifted in), then the four
// row minima are combined on the scalar unit.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
  const uint32_t I = 0xffffffffu;  // identity of unsigned min
  v = min(v, row_shr<1>(I, v));
  v = min(v, row_shr<2>(I, v));
  v = min(v, row_shr<4>(I, v));
  v = min(v, row_shr<8>(I, v));
  const uint32_t r0 = rdlane(v, 15), r1 = rdlane(v, 31), r2 = rdlane(v, 47), r3 = rdlane(v, 63);
  return min(min(r0, r1), min(r2, r3));
}

__device__ __forceinline__ uint32_t floor_log2_u32(uint32_t x) {  // x >= 1
  return 31u - (uint32_t)__builtin_clz(x);
}
__device__ __forceinline__ uint32_t ceil_log2_u32(uint32_t x) {   // x >= 1
  return x <= 1u ? 0u : 32u - (uint32_t)__builtin_clz(x - 1u);
}

// A table entry packs a block as (size << 32) | address, both in granules,
// so that comparing entries compares (size, address) lexicographically.
typedef uint64_t Ent;
__device__ __forceinline__ Ent mk_ent(uint32_t a, uint32_t s) { return ((uint64_t)s << 32) | a; }
__device__ __forceinline__ uint32_t ent_a(Ent e) { return (uint32_t)e; }
__device__ __forceinline__ uint32_t ent_s(Ent e) { return (uint32_t)(e >> 32); }

// Where a heap's tables live.
struct Tables {
  HDA_LDS Ent* lf;           // LDS free entries [0, kf)
  HDA_LDS uint32_t* lst;     // LDS stamps       [0, kf)
  HDA_LDS Ent* ll;           // LDS live entries [0, kl)
  HDA_GLOBAL Ent* gf;        // device free entries [kf, cf), indexed from 0
  HDA_GLOBAL uint32_t* gst;  // device stamps       [kf, cf)
  HDA_GLOBAL Ent* gl;        // device live entries [kl, cl)
  uint32_t kf, kl;           // LDS capacities (multiples of 64)
  uint32_t cf, cl;           // total capacities (multiples of 64)
};

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

// ---- table access (index wave-uniform for single entries) ----
__device__ __forceinline__ Ent fget(const Tables& t, uint32_t i) {
  wave_sync();
  if (i < t.kf) return t.lf[i];
  return t.gf[i - t.kf];
}
__device__ __forceinline__ void fset(const Tables& t, uint32_t i, Ent e) {
  wave_sync();
  if (lane_id() == 0) {
    if (i < t.kf) t.lf[i] = e; else t.gf[i - t.kf] = e;
  }
}
__device__ __forceinline__ uint32_t sget(const Tables& t, uint32_t i) {
  wave_sync();
  if (i < t.kf) return t.lst[i];
  return t.gst[i - t.kf];
}
__device__ __forceinline__ void sset(const Tables& t, uint32_t i, uint32_t s) {
  wave_sync();
  if (lane_id() == 0) {
    if (i < t.kf) t.lst[i] = s; else t.gst[i - t.kf] = s;
  }
}
__device__ __forceinline__ Ent lget(const Tables& t, uint32_t i) {
  wave_sync();
  if (i < t.kl) return t.ll[i];
  return t.gl[i - t.kl];
}
__device__ __forceinline__ void lset(const Tables& t, uint32_t i, Ent e) {
  wave_sync();
  if (lane_id() == 0) {
    if (i < t.kl) t.ll[i] = e; else t.gl[i - t.kl] = e;
  }
}
// chunk loads: `base` is wave-uniform and a multiple of 64
__device__ __forceinline__ Ent fchunk(const Tables& t, uint32_t base) {
  wave_sync();
  if (base < t.kf) return t.lf[base + lane_id()];
  return t.gf[base - t.kf + lane_id()];
}
__device__ __forceinline__ uint32_t schunk(const Tables& t, uint32_t base) {
  wave_sync();
  if (base < t.kf) return t.lst[base + lane_id()];
  return t.gst[base - t.kf + lane_id()];
}
__device__ __forceinline__ Ent lchunk(const Tables& t, uint32_t base) {
  wave_sync();
  if (base < t.kl) return t.ll[base + lane_id()];
  return t.gl[base - t.kl + lane_id()];
}

// Byte class of a free block of `sg` granules.
__device__ __forceinline__ uint32_t byte_class(const HeapRegs& h, uint32_t sg) {
  return floor_log2_u32(sg) + h.shift;
}

__device__ __forceinline__ void cnt_add(HeapRegs& h, uint32_t cls, int d) {
  h.cnt += (lane_id() == cls) ? (uint32_t)d : 0u;
}

__device__ __forceinline__ uint64_t class_bitmap(const HeapRegs& h) {
  return ballot(h.cnt != 0u);
}

// Alg. 6: the free table starts as one block [0, A).
__device__ __forceinline__ void heap_init(const Tables& t, HeapRegs& h) {
  h.F = 1;
  h.L = 0;
  h.rover = 0;
  h.clock = 1;
  h.cnt = 0;
  fset(t, 0, mk_ent(0u, h.ag));
  sset(t, 0, h.clock++);  // stamps start at 1: the search key ~stamp never equals kNone
  cnt_add(h, byte_class(h, h.ag), 1);
}

// Remove free entry j: the last entry moves into its place.
__device__ __forceinline__ void free_remove(const Tables& t, HeapRegs& h, uint32_t j) {
  const uint32_t last = h.F - 1u;
  if (j != last) {
    fset(t, j, fget(t, last));
    if (h.algo == kSegFit) sset(t, j, sget(t, last));
  }
  h.F = last;
}

// Selection (Sec. II, Sec. IV, Sec. V-A).  Returns the chosen entry's index or
// kNone; *e_out receives the entry.
__device__ uint32_t select_block(const Tables& t, const HeapRegs& h, uint32_t sg,
                                 uint32_t seg_class, Ent* e_out) {
  const uint32_t lane = lane_id();
  const Ent need = (uint64_t)sg << 32;   // e >= need  <=>  size >= sg
  // lane-local best: 32-bit primary key k1 (and k2 for best fit), its entry
  // index and the entry itself
  uint32_t k1 = kNone, k2 = kNone, bi = kNone;
  Ent be = 0;
  // next fit keeps a second candidate for the wrapped tier
  uint32_t w1 = kNone, wi = kNone;
  Ent we = 0;
  const int algo = h.algo;
  const uint32_t seg_lo = (algo == kSegFit) ? seg_class - h.shift : 0u;
  for (uint32_t base = 0; base < h.F; base += 64u) {
    const uint32_t i = base + lane;
    const bool v = i < h.F;
    const Ent e = fchunk(t, base);
    const uint32_t a = ent_a(e), s = ent_s(e);
    // lane-local updates are selects, not branches: their results feed the
    // wave-wide reductions below
    if (algo == kFirstFit) {
      const bool take = v && e >= need && a < k1;
      k1 = take ? a : k1; bi = take ? i : bi; be = take ? e : be;
    } else if (algo == kBestFit) {
      const bool take = v && e >= need && (s < k1 || (s == k1 && a < k2));
      k1 = take ? s : k1; k2 = take ? a : k2; bi = take ? i : bi; be = take ? e : be;
    } else if (algo == kNextFit) {
      const bool fit = v && e >= need;
      const bool past = a + s > h.rover;
      const bool take = fit && past && a < k1;
      const bool wrap = fit && !past && a < w1;
      k1 = take ? a : k1; bi = take ? i : bi; be = take ? e : be;
      w1 = wrap ? a : w1; wi = wrap ? i : wi; we = wrap ? e : we;
    } else {  // segregated fit: the class-c block pushed last
      const uint32_t st = schunk(t, base);
      const bool take = v && (s >> seg_lo) == 1u && ~st < k1;
      k1 = take ? ~st : k1; bi = take ? i : bi; be = take ? e : be;
    }
  }
  uint32_t K = wave_min(k1);
  if (algo == kNextFit && K == kNone) {  // nothing past the rover: wrap around
    k1 = w1; bi = wi; be = we;
    K = wave_min(k1);
  }
  if (K == kNone) return kNone;
  uint64_t m;
  if (algo == kBestFit) {
    const uint32_t A2 = wave_min(k1 == K ? k2 : kNone);
    m = ballot(k1 == K && k2 == A2);
  } else {
    m = ballot(k1 == K);
  }
  const uint32_t wl = (uint32_t)__builtin_ctzll(m);
  *e_out = mk_ent(rdlane(ent_a(be), wl), rdlane(ent_s(be), wl));
  return rdlane(bi, wl);
}

// One allocation request of `q` bytes (q >= 0).  Returns the byte offset, -1,
// or kENoMeta (state unchanged).
__device__ int64_t op_alloc(const Tables& t, HeapRegs& h, int64_t q) {
  if (q > h.arena) return kFail;
  const uint64_t gm = (1ull << h.shift) - 1ull;
  uint32_t sg = (uint32_t)(((uint64_t)q + gm) >> h.shift);
  if (sg == 0u) sg = 1u;
  uint32_t c = 0;
  if (h.algo == kSegFit) {
    const uint32_t k = ceil_log2_u32(sg) + h.shift;  // request class (Sec. V-A)
    if (k >= 64u) return kFail;
    const uint64_t m = class_bitmap(h) & (~0ull << k);
    if (m == 0ull) return kFail;
    c = (uint32_t)__builtin_ctzll(m);
  }
  Ent e;
  const uint32_t j = select_block(t, h, sg, c, &e);
  if (j == kNone) return kFail;
  if (h.L >= t.cl) return kENoMeta;
  const uint32_t a = ent_a(e), bs = ent_s(e);
  if (bs > sg) {                        // Alg. 1 / Alg. 4: keep the high remainder
    fset(t, j, mk_ent(a + sg, bs - sg));
    if (h.algo == kSegFit) {
      sset(t, j, h.clock++);
      cnt_add(h, byte_class(h, bs), -1);
      cnt_add(h, byte_class(h, bs - sg), 1);
    }
  } else {
    free_remove(t, h, j);
    if (h.algo == kSegFit) cnt_add(h, byte_class(h, bs), -1);
  }
  lset(t, h.L, mk_ent(a, sg));
  h.L++;
  if (h.algo == kNextFit) h.rover = a + sg;
  return (int64_t)((uint64_t)a << h.shift);
}

// Release block [x, x+sz) (granules) into the free table, merging with free
// neighbours (Alg. 2 / Alg. 5).  Returns false (nothing changed) when the
// free table is full and a new entry would be needed.
__device__ bool release_block(const Tables& t, HeapRegs& h, uint32_t x, uint32_t sz) {
  const uint32_t lane = lane_id();
  const uint32_t xe = x + sz;
  uint32_t jl = kNone, jr = kNone, sl = 0, sr = 0;
  for (uint32_t base = 0; base < h.F; base += 64u) {
    const bool v = base + lane < h.F;
    const Ent e = fchunk(t, base);
    const uint32_t a = ent_a(e), s = ent_s(e);
    const uint64_t ml = ballot(v && a + s == x);
    const uint64_t mr = ballot(v && a == xe);
    if (ml) { const uint32_t w = (uint32_t)__builtin_ctzll(ml); jl = base + w; sl = rdlane(s, w); }
    if (mr) { const uint32_t w = (uint32_t)__builtin_ctzll(mr); jr = base + w; sr = rdlane(s, w); }
  }
  const bool seg = h.algo == kSegFit;
  if (jl == kNone && jr == kNone) {
    if (h.F >= t.cf) return false;
    fset(t, h.F, mk_ent(x, sz));
    if (seg) { sset(t, h.F, h.clock++); cnt_add(h, byte_class(h, sz), 1); }
    h.F++;
  } else if (jr == kNone) {
    fset(t, jl, mk_ent(x - sl, sl + sz));
    if (seg) {
      sset(t, jl, h.clock++);
      cnt_add(h, byte_class(h, sl), -1);
      cnt_add(h, byte_class(h, sl + sz), 1);
    }
  } else if (jl == kNone) {
    fset(t, jr, mk_ent(x, sz + sr));
    if (seg) {
      sset(t, jr, h.clock++);
      cnt_add(h, byte_class(h, sr), -1);
      cnt_add(h, byte_class(h, sz + sr), 1);
    }
  } else {
    const uint32_t ms = sl + sz + sr;
    const uint32_t last = h.F - 1u;
    uint32_t keep;                       // slot that ends up holding the merged block
    if (jr == last) {
      keep = jl;
    } else if (jl == last) {
      keep = jr;
    } else {
      keep = jl;
      fset(t, jr, fget(t, last));
      if (seg) sset(t, jr, sget(t, last));
    }
    fset(t, keep, mk_ent(x - sl, ms));
    if (seg) {
      sset(t, keep, h.clock++);
      cnt_add(h, byte_class(h, sl), -1);
      cnt_add(h, byte_class(h, sr), -1);
      cnt_add(h, byte_class(h, ms), 1);
    }
    h.F = last;
  }
  return true;
}

// Free the live block at live-table index idx.  Returns its byte offset or
// kENoMeta (state unchanged).
__device__ int64_t op_free_index(const Tables& t, HeapRegs& h, uint32_t idx) {
  const Ent b = lget(t, idx);
  if (!release_block(t, h, ent_a(b), ent_s(b))) return kENoMeta;
  const uint32_t last = h.L - 1u;
  if (idx != last) lset(t, idx, lget(t, last));
  h.L = last;
  return (int64_t)((uint64_t)ent_a(b) << h.shift);
}

// Replay-driver free: r = ~q is the 32-bit draw, the victim is
// live[(r * L) >> 32]; nothing live -> -1.
__device__ __forceinline__ int64_t op_free_draw(const Tables& t, HeapRegs& h, int64_t q) {
  if (h.L == 0u) return kFail;
  const uint32_t r = (uint32_t)~(uint64_t)q;
  const uint32_t idx = (uint32_t)(((uint64_t)r * (uint64_t)h.L) >> 32);
  return op_free_index(t, h, idx);
}

// Free by byte offset (the call-by-call interface): find the live entry.
__device__ int64_t op_free_offset(const Tables& t, HeapRegs& h, int64_t off) {
  const uint64_t gm = (1ull << h.shift) - 1ull;
  if (off < 0 || off >= h.arena || ((uint64_t)off & gm)) return kEBadFree;
  const uint32_t x = (uint32_t)((uint64_t)off >> h.shift);
  uint32_t idx = kNone;
  for (uint32_t base = 0; base < h.L && idx == kNone; base += 64u) {
    const bool v = base + lane_id() < h.L;
    const Ent e = lchunk(t, base);
    const uint64_t m = ballot(v && ent_a(e) == x);
    if (m) idx = base + (uint32_t)__builtin_ctzll(m);
  }
  if (idx == kNone) return kEBadFree;
  const int64_t r = op_free_index(t, h, idx);
  return r < 0 ? r : 0;
}

__device__ __forceinline__ int64_t op_request(const Tables& t, HeapRegs& h, int64_t q) {
  return q >= 0 ? op_alloc(t, h, q) : op_free_draw(t, h, q);
}

// Canonical state (format in hda.h), written by the whole wave.  The free
// table is ranked by address and, for segregated fit, by descending stamp
// within each class.  Returns the number of words (written only if <= cap).
__device__ int64_t dump_state(const Tables& t, const HeapRegs& h, int64_t* out, int64_t cap) {
  const uint32_t lane = lane_id();
  const bool seg = h.algo == kSegFit;
  const int64_t need = 4 + 2 * (int64_t)h.F + 2 * (int64_t)h.L + (seg ? 64 + (int64_t)h.F : 0);
  if (out == nullptr || need > cap) return need;
  const uint32_t sh = h.shift;
  if (lane == 0) out[0] = h.F;
  int64_t* fo = out + 1;
  for (uint32_t base = 0; base < h.F; base += 64u) {
    const uint32_t i = base + lane;
    const bool v = i < h.F;
    const Ent e = fchunk(t, base);
    uint32_t rank = 0;
    for (uint32_t j = 0; j < h.F; ++j) rank += ent_a(fget(t, j)) < ent_a(e) ? 1u : 0u;
    if (v) {
      fo[2 * rank] = (int64_t)((uint64_t)ent_a(e) << sh);
      fo[2 * rank + 1] = (int64_t)((uint64_t)ent_s(e) << sh);
    }
  }
  int64_t* lo = out + 1 + 2 * (int64_t)h.F;
  if (lane == 0) lo[0] = h.L;
  for (uint32_t base = 0; base < h.L; base += 64u) {
    const uint32_t i = base + lane;
    const Ent e = lchunk(t, base);
    if (i < h.L) {
      lo[1 + 2 * i] = (int64_t)((uint64_t)ent_a(e) << sh);
      lo[2 + 2 * i] = (int64_t)((uint64_t)ent_s(e) << sh);
    }
  }
  int64_t* tail = lo + 1 + 2 * (int64_t)h.L;
  const uint64_t bm = class_bitmap(h);
  if (lane == 0) {
    tail[0] = h.algo == kNextFit ? (int64_t)((uint64_t)h.rover << sh) : -1;
    tail[1] = seg ? (int64_t)bm : 0;
  }
  if (seg) {
    int64_t* ls = tail + 2;
    // header position of class `lane`: sum over lower classes of (1 + count)
    uint32_t hdr = 0, acc = 0;
    for (uint32_t c = 0; c < 64u; ++c) {
      hdr = (lane == c) ? acc : hdr;
      acc += 1u + rdlane(h.cnt, c);
    }
    const uint32_t region = 64u + h.F;   // words of the class-list section
    if (hdr < region) ls[hdr] = h.cnt;
    for (uint32_t base = 0; base < h.F; base += 64u) {
      const uint32_t i = base + lane;
      const bool v = i < h.F;
      const Ent e = fchunk(t, base);
      const uint32_t st = schunk(t, base);
      const uint32_t c = v ? byte_class(h, ent_s(e)) : 0u;
      uint32_t rank = 0;
      for (uint32_t j = 0; j < h.F; ++j) {
        const uint32_t fs = ent_s(fget(t, j));
        const uint32_t sj = sget(t, j);
        rank += (fs != 0u && byte_class(h, fs) == c && sj > st) ? 1u : 0u;
      }
      const uint32_t hc = shfl(hdr, c);
      if (v && hc + 1u + rank < region) ls[hc + 1u + rank] = (int64_t)((uint64_t)ent_a(e) << sh);
    }
  }
  return need;
}

}  // namespace hda
