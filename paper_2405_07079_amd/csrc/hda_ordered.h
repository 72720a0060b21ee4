// Ordered replay core: one wavefront replays one heap with its free blocks
// kept in address order, so that every step of Alg. 1-5 costs a fixed number
// of wave operations however many free blocks the heap has.
//
// Free blocks form a sorted array of 64-entry chunks, one entry per lane --
// the hybrid array list of App. A, whose traversal costs O(n/m + m) on one
// CPU thread.  Here a directory held in D VGPRs replaces the walk over the
// chunk list: lane l of directory register v describes chunk 64 v + l in
// address order (its storage slot, its number of entries, its first key and,
// for first and next fit, the largest block in it).  Finding the chunk that
// holds an address, or the first chunk holding a block of at least s
// granules, is one ballot per directory register; finding the entry inside
// it is one chunk load and one ballot.  A full chunk splits into 33 + 32
// entries; a chunk that drops below 32 entries merges with a neighbour or
// takes entries from it.  So while there are two or more chunks each holds at
// least 32 entries, and the directory's 64 D chunks always hold 2,048 D free
// blocks.
//
// Per algorithm:
//  * first fit (Sec. II-A): the first chunk whose largest block fits, then
//    the first fitting entry in it.
//  * next fit (Sec. II-A, Sec. IV): the block holding the rover or the next
//    one is located like an address; the search runs on from there through
//    the directory and wraps once.
//  * best fit (Alg. 3): a second sorted chunk table holds the keys
//    (size, address); the smallest key at or above (s, 0) is the best fit.
//  * segregated fit (Alg. 4-5) and TLSF (Sec. V-B): each free entry carries
//    the class-list links of Alg. 4-5 (next and previous block, by address,
//    NIL = kNone), the list heads sit in a VGPR (segregated fit: lane k heads
//    class k) or in LDS (TLSF's 2,048 classes), and the availability bitmaps
//    are a scalar (segregated fit; TLSF's first level) and a VGPR (TLSF's
//    second level: lane fl holds the 32 sub-class bits of level fl).  The
//    paper's address-keyed hash lookup ht[addr] becomes a lookup in the
//    address-ordered table; the block ending at a freed block and the one
//    after it are its neighbours in that order (no prev_adj field needed).
//
// Results equal those of the other cores and the oracle: selection,
// splitting, merging and the class lists follow the same definitions.
//
// Storage: chunk slots and live entries below the LDS counts given at
// construction are in the wave's LDS pool, the rest in its device-memory
// slot.  Every memory access is preceded by wave_sync() (a no-op on the GPU;
// the CPU wave emulation switches lanes there).  As in the other cores,
// values that feed a cross-lane operation are never produced under a
// lane-dependent branch, and every entry write is done by all lanes with the
// same value.
#pragma once
#include <stdint.h>

#include "hda_core.h"

namespace hda {

// 8- and 16-byte entries as plain vectors (loaded and stored whole through
// pointers of any address space).
typedef uint32_t u32x2 __attribute__((vector_size(8)));
typedef uint32_t u32x4 __attribute__((vector_size(16)));

// Wave-wide maximum of a u32 (every lane active).
__device__ __forceinline__ uint32_t wave_max(uint32_t v) { return ~wave_min(~v); }

// Directory access: lane (i & 63) of register i >> 6.
template <int D>
__device__ __forceinline__ uint32_t dir_get(const uint32_t (&v)[D], uint32_t i) {
  uint32_t x = rdlane(v[0], i & 63u);
#pragma unroll
  for (int k = 1; k < D; ++k) {
    const uint32_t y = rdlane(v[k], i & 63u);
    x = (i >> 6) == (uint32_t)k ? y : x;
  }
  return x;
}
template <int D>
__device__ __forceinline__ void dir_put(uint32_t (&v)[D], uint32_t i, uint32_t x) {
  const bool me = lane_id() == (i & 63u);
#pragma unroll
  for (int k = 0; k < D; ++k) v[k] = (me && (i >> 6) == (uint32_t)k) ? x : v[k];
}
// Open a hole at directory position i (entries i.. move up by one; the last
// one falls off) and put x there.
template <int D>
__device__ __forceinline__ void dir_insert(uint32_t (&v)[D], uint32_t i, uint32_t x) {
  const uint32_t lane = lane_id();
  uint32_t carry = x;  // lane 63 of the register below, before the shift
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const uint32_t top = rdlane(v[k], 63);
    const uint32_t up = shfl(v[k], lane == 0u ? 0u : lane - 1u);
    const uint32_t g = 64u * (uint32_t)k + lane;
    const uint32_t moved = lane == 0u ? carry : up;
    v[k] = g > i ? moved : (g == i ? x : v[k]);
    carry = top;
  }
}
// Remove directory position i (entries past it move down); the last
// position receives `fill`.
template <int D>
__device__ __forceinline__ void dir_erase(uint32_t (&v)[D], uint32_t i, uint32_t fill) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const uint32_t next0 = k + 1 < D ? rdlane(v[k + 1 < D ? k + 1 : k], 0) : fill;
    const uint32_t down = shfl(v[k], lane == 63u ? 63u : lane + 1u);
    const uint32_t g = 64u * (uint32_t)k + lane;
    const uint32_t moved = lane == 63u ? next0 : down;
    v[k] = g >= i ? moved : v[k];
  }
}

// One table of sorted chunks.  REC: 16-byte entries (address, size, next,
// prev) instead of 8-byte ones (address, size).  KEY64: sorted by (size,
// address) instead of by address.  MAXS: the directory keeps each chunk's
// largest size.
template <bool REC, bool KEY64, bool MAXS, int D>
struct Hal {
  static constexpr uint32_t NC = 64u * D;         // chunk slots
  static constexpr uint32_t EB = REC ? 16u : 8u;  // bytes per entry
  static constexpr uint32_t CB = 64u * EB;        // bytes per chunk

  // this lane's entry of a loaded chunk; positions past the chunk's count
  // hold the sentinel (address kNone, size 0, or size kNone when sorted by
  // size), which sorts after every real entry and fits no request
  struct Row {
    uint32_t a, s, nx, pv;
  };

  HDA_LDS uint8_t* lb;     // slots [0, nl) in LDS
  HDA_GLOBAL uint8_t* gb;  // slot i >= nl at gb + i * CB in device memory
  uint32_t nl;
  uint32_t dsl[D], dct[D], dk0[D], dk1[D], dmx[D];  // slot, count, first key, max size
  uint64_t used[D];                                 // slots in use
  uint32_t nc;                                      // chunks

  static constexpr uint32_t kSentS = KEY64 ? kNone : 0u;

  __device__ __forceinline__ static Row sentinel() { return Row{kNone, kSentS, kNone, kNone}; }

  __device__ __forceinline__ void init(HDA_LDS uint8_t* l, HDA_GLOBAL uint8_t* g, uint32_t n_lds) {
    lb = l;
    gb = g;
    nl = n_lds < NC ? n_lds : NC;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      dsl[k] = 0u; dct[k] = 0u; dk0[k] = kNone; dk1[k] = kNone; dmx[k] = 0u;
      used[k] = 0ull;
    }
    nc = 0;
  }

  // ---- chunk memory ----
  __device__ __forceinline__ Row load(uint32_t sl) const {
    wave_sync();
    sl = sl < NC ? sl : NC - 1u;  // (slot ids are below NC; kept in the table)
    const uint32_t lane = lane_id();
    Row r;
    if constexpr (REC) {
      u32x4 v;
      if (sl < nl) v = *(const HDA_LDS u32x4*)(lb + sl * CB + lane * 16u);
      else v = *(const HDA_GLOBAL u32x4*)(gb + (uint64_t)sl * CB + lane * 16u);
      r.a = v[0]; r.s = v[1]; r.nx = v[2]; r.pv = v[3];
    } else {
      u32x2 v;
      if (sl < nl) v = *(const HDA_LDS u32x2*)(lb + sl * CB + lane * 8u);
      else v = *(const HDA_GLOBAL u32x2*)(gb + (uint64_t)sl * CB + lane * 8u);
      r.a = v[0]; r.s = v[1]; r.nx = kNone; r.pv = kNone;
    }
    return r;
  }
  __device__ __forceinline__ void store(uint32_t sl, const Row& r) const {
    wave_sync();
    sl = sl < NC ? sl : NC - 1u;  // (slot ids are below NC; kept in the table)
    const uint32_t lane = lane_id();
    if constexpr (REC) {
      u32x4 v;
      v[0] = r.a; v[1] = r.s; v[2] = r.nx; v[3] = r.pv;
      if (sl < nl) *(HDA_LDS u32x4*)(lb + sl * CB + lane * 16u) = v;
      else *(HDA_GLOBAL u32x4*)(gb + (uint64_t)sl * CB + lane * 16u) = v;
    } else {
      u32x2 v;
      v[0] = r.a; v[1] = r.s;
      if (sl < nl) *(HDA_LDS u32x2*)(lb + sl * CB + lane * 8u) = v;
      else *(HDA_GLOBAL u32x2*)(gb + (uint64_t)sl * CB + lane * 8u) = v;
    }
  }
  // one 32-bit field (0 address, 1 size, 2 next, 3 prev) of entry p, written
  // by every lane with the same value
  __device__ __forceinline__ void store_field(uint32_t sl, uint32_t p, uint32_t f,
                                              uint32_t x) const {
    wave_sync();
    sl = sl < NC ? sl : NC - 1u;
    const uint32_t off = (p & 63u) * EB + (f & 3u) * 4u;
    if (sl < nl) *(HDA_LDS uint32_t*)(lb + sl * CB + off) = x;
    else *(HDA_GLOBAL uint32_t*)(gb + (uint64_t)sl * CB + off) = x;
  }
  __device__ __forceinline__ void store_entry(uint32_t sl, uint32_t p, uint32_t a, uint32_t s,
                                              uint32_t nx, uint32_t pv) const {
    wave_sync();
    p &= 63u;  // (positions are below 64; the mask keeps every store in its chunk)
    sl = sl < NC ? sl : NC - 1u;
    if constexpr (REC) {
      u32x4 v;
      v[0] = a; v[1] = s; v[2] = nx; v[3] = pv;
      if (sl < nl) *(HDA_LDS u32x4*)(lb + sl * CB + p * 16u) = v;
      else *(HDA_GLOBAL u32x4*)(gb + (uint64_t)sl * CB + p * 16u) = v;
    } else {
      u32x2 v;
      v[0] = a; v[1] = s;
      if (sl < nl) *(HDA_LDS u32x2*)(lb + sl * CB + p * 8u) = v;
      else *(HDA_GLOBAL u32x2*)(gb + (uint64_t)sl * CB + p * 8u) = v;
    }
  }

  // ---- keys ----
  __device__ __forceinline__ static bool row_le(const Row& r, uint32_t k1, uint32_t k0) {
    return KEY64 ? (r.s < k1 || (r.s == k1 && r.a <= k0)) : r.a <= k0;
  }
  __device__ __forceinline__ static bool row_lt(const Row& r, uint32_t k1, uint32_t k0) {
    return KEY64 ? (r.s < k1 || (r.s == k1 && r.a < k0)) : r.a < k0;
  }
  // chunks whose first key is <= (k1, k0) (strict: <)
  __device__ __forceinline__ uint32_t count_first(uint32_t k1, uint32_t k0, bool strict) const {
    uint32_t n = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const uint32_t g = 64u * (uint32_t)k + lane_id();
      const bool le = KEY64 ? (dk1[k] < k1 || (dk1[k] == k1 && (strict ? dk0[k] < k0 : dk0[k] <= k0)))
                            : (strict ? dk0[k] < k0 : dk0[k] <= k0);
      n += (uint32_t)__builtin_popcountll(ballot(g < nc && le));
    }
    return n;
  }

  __device__ __forceinline__ uint32_t slot(uint32_t ci) const { return dir_get(dsl, ci); }
  __device__ __forceinline__ uint32_t count(uint32_t ci) const { return dir_get(dct, ci); }

  // Directory entry of chunk ci from its loaded row (n entries).
  __device__ __forceinline__ void describe(uint32_t ci, const Row& r, uint32_t n) {
    dir_put(dct, ci, n);
    dir_put(dk0, ci, rdlane(r.a, 0));
    if (KEY64) dir_put(dk1, ci, rdlane(r.s, 0));
    if (MAXS) dir_put(dmx, ci, wave_max(r.s));
  }

  __device__ __forceinline__ uint32_t take_slot() {
    uint32_t s = kNone;
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
      const uint64_t fr = ~used[k];
      s = fr != 0ull ? 64u * (uint32_t)k + ctz64(fr) : s;
    }
    // the occupancy rule leaves a free slot whenever a chunk is added; the
    // last slot stands in should that ever fail, so no access leaves the table
    s = s == kNone ? NC - 1u : s;
#pragma unroll
    for (int k = 0; k < D; ++k)
      used[k] |= (s >> 6) == (uint32_t)k ? 1ull << (s & 63u) : 0ull;
    return s;
  }
  __device__ __forceinline__ void drop_slot(uint32_t s) {
#pragma unroll
    for (int k = 0; k < D; ++k)
      used[k] &= (s >> 6) == (uint32_t)k ? ~(1ull << (s & 63u)) : ~0ull;
  }

  // A table holding one entry.
  __device__ __forceinline__ void start(uint32_t a, uint32_t s, uint32_t nx, uint32_t pv) {
    const uint32_t sl = take_slot();
    Row r = sentinel();
    const bool me = lane_id() == 0u;
    r.a = me ? a : r.a; r.s = me ? s : r.s; r.nx = me ? nx : r.nx; r.pv = me ? pv : r.pv;
    store(sl, r);
    nc = 1;
    dir_put(dsl, 0u, sl);
    describe(0u, r, 1u);
  }

  // Row shifted: lane l receives lane src(l) of r (or the sentinel when the
  // source is out of range).
  __device__ __forceinline__ static Row pull(const Row& r, uint32_t src, bool ok) {
    Row o;
    const uint32_t s = src & 63u;
    o.a = shfl(r.a, s); o.s = shfl(r.s, s);
    if (REC) { o.nx = shfl(r.nx, s); o.pv = shfl(r.pv, s); } else { o.nx = o.pv = kNone; }
    const Row z = sentinel();
    o.a = ok ? o.a : z.a; o.s = ok ? o.s : z.s; o.nx = ok ? o.nx : z.nx; o.pv = ok ? o.pv : z.pv;
    return o;
  }
  __device__ __forceinline__ static Row pick(bool c, const Row& x, const Row& y) {
    Row o;
    o.a = c ? x.a : y.a; o.s = c ? x.s : y.s; o.nx = c ? x.nx : y.nx; o.pv = c ? x.pv : y.pv;
    return o;
  }

  // Insert entry e at position p (0 <= p <= count) of chunk ci, whose row r
  // has just been loaded.  The caller guarantees order and capacity.
  __device__ __forceinline__ void insert_at(uint32_t ci, uint32_t p, const Row& r, const Row& e) {
    const uint32_t lane = lane_id();
    const uint32_t n = count(ci), sl = slot(ci);
    if (n < 64u) {
      const Row up = pull(r, lane - 1u, lane >= 1u);
      const Row o = pick(lane < p, r, pick(lane == p, e, up));
      store(sl, o);
      describe(ci, o, n + 1u);
      return;
    }
    // split: the 65 entries c[0..64] become 33 here and 32 in a new chunk
    // after it; c[i] = r[i] (i < p), e (i == p), r[i - 1] (i > p)
    const uint32_t ns = take_slot();
    const Row lo_up = pull(r, lane - 1u, lane >= 1u);
    Row left = pick(lane < p, r, pick(lane == p, e, lo_up));
    left = pick(lane <= 32u, left, sentinel());
    const uint32_t i = lane + 33u;  // position in c of this lane's right entry
    const Row r_same = pull(r, i, i < 64u);
    const Row r_prev = pull(r, i - 1u, true);
    Row right = pick(i < p, r_same, pick(i == p, e, r_prev));
    right = pick(lane < 32u, right, sentinel());
    store(sl, left);
    store(ns, right);
    describe(ci, left, 33u);
    dir_insert(dsl, ci + 1u, ns);
    dir_insert(dct, ci + 1u, 32u);
    dir_insert(dk0, ci + 1u, rdlane(right.a, 0));
    if (KEY64) dir_insert(dk1, ci + 1u, rdlane(right.s, 0));
    if (MAXS) dir_insert(dmx, ci + 1u, wave_max(right.s));
    ++nc;
  }

  // Remove the entry at position p of chunk ci (row r just loaded), then
  // keep every chunk at 32 entries or more while there are two or more.
  __device__ __forceinline__ void erase_at(uint32_t ci, uint32_t p, const Row& r) {
    const uint32_t lane = lane_id();
    const uint32_t n = count(ci) - 1u, sl = slot(ci);
    const Row down = pull(r, lane + 1u, lane < 63u);
    const Row o = pick(lane >= p, down, r);
    if (n >= 32u || nc == 1u) {
      store(sl, o);
      describe(ci, o, n);
      return;
    }
    // join with the next chunk (or the previous one for the last chunk)
    const uint32_t lo = ci + 1u < nc ? ci : ci - 1u, hi = lo + 1u;
    const uint32_t sl_lo = slot(lo), sl_hi = slot(hi);
    const Row other = load(ci == lo ? sl_hi : sl_lo);
    const Row L = ci == lo ? o : other, H = ci == lo ? other : o;
    const uint32_t nL = ci == lo ? n : count(lo), nH = ci == lo ? count(hi) : n;
    const uint32_t T = nL + nH;
    // c[i] = L[i] (i < nL), H[i - nL] (i >= nL)
    if (T <= 64u) {
      const Row hp = pull(H, lane - nL, lane >= nL && lane < T);
      const Row m = pick(lane < nL, L, hp);
      store(sl_lo, m);
      describe(lo, m, T);
      drop_slot(sl_hi);
      dir_erase(dsl, hi, 0u);
      dir_erase(dct, hi, 0u);
      dir_erase(dk0, hi, kNone);
      if (KEY64) dir_erase(dk1, hi, kNone);
      if (MAXS) dir_erase(dmx, hi, 0u);
      --nc;
      return;
    }
    // share the T (65..95) entries: T / 2 in the lower chunk, the rest above
    const uint32_t a = T >> 1, b = T - a;
    const Row hp = pull(H, lane - nL, lane >= nL);
    Row m0 = pick(lane < nL, L, hp);
    m0 = pick(lane < a, m0, sentinel());
    const uint32_t i = lane + a;
    const Row lsrc = pull(L, i, i < nL);
    const Row hsrc = pull(H, i - nL, i >= nL && i < T);
    Row m1 = pick(i < nL, lsrc, hsrc);
    m1 = pick(lane < b, m1, sentinel());
    store(sl_lo, m0);
    store(sl_hi, m1);
    describe(lo, m0, a);
    describe(hi, m1, b);
  }

  // The chunk holding key (k1, k0) or the last chunk whose first key is
  // below it: ci (kNone if every chunk starts above it), its row, and p =
  // the position of the last entry <= the key (kNone if none).
  __device__ __forceinline__ void locate(uint32_t k1, uint32_t k0, uint32_t& ci, Row& r,
                                         uint32_t& p) const {
    const uint32_t c = count_first(k1, k0, false);
    if (c == 0u) { ci = kNone; p = kNone; return; }
    ci = c - 1u;
    r = load(slot(ci));
    const uint32_t n = count(ci);
    p = (uint32_t)__builtin_popcountll(ballot(lane_id() < n && row_le(r, k1, k0))) - 1u;
  }
  // Where a new key goes: chunk ci (the last one starting below it, else
  // the first), its row, and the position of the first entry above it.
  __device__ __forceinline__ void insert_pos(uint32_t k1, uint32_t k0, uint32_t& ci, Row& r,
                                             uint32_t& p) const {
    const uint32_t c = count_first(k1, k0, true);
    ci = c == 0u ? 0u : c - 1u;
    r = load(slot(ci));
    const uint32_t n = count(ci);
    p = (uint32_t)__builtin_popcountll(ballot(lane_id() < n && row_lt(r, k1, k0)));
  }
  __device__ __forceinline__ void insert_key(uint32_t a, uint32_t s) {
    uint32_t ci, p;
    Row r;
    insert_pos(s, a, ci, r, p);
    Row e = sentinel();
    e.a = a; e.s = s;
    insert_at(ci, p, r, e);
  }
  __device__ __forceinline__ void erase_key(uint32_t a, uint32_t s) {
    uint32_t ci, p;
    Row r;
    locate(s, a, ci, r, p);
    erase_at(ci, p, r);
  }
  // first chunk at or after `from` whose largest block has >= sg granules
  // (MAXS tables), or kNone
  __device__ __forceinline__ uint32_t first_fit_chunk(uint32_t sg, uint32_t from) const {
    uint32_t c = kNone;
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
      const uint32_t g = 64u * (uint32_t)k + lane_id();
      const uint64_t m = ballot(g < nc && g >= from && dmx[k] >= sg);
      c = m != 0ull ? 64u * (uint32_t)k + ctz64(m) : c;
    }
    return c;
  }
};

// Where one heap's tables live.  Table slots and live entries below the LDS
// counts are in the wave's LDS pool; the others are in its device slot.
struct OrdMem {
  HDA_LDS uint8_t* ta_l;
  HDA_GLOBAL uint8_t* ta_g;
  uint32_t ta_n;
  HDA_LDS uint8_t* tb_l;
  HDA_GLOBAL uint8_t* tb_g;
  uint32_t tb_n;
  HDA_LDS Ent* ll;
  HDA_GLOBAL Ent* gl;
  uint32_t ll_n;
  HDA_LDS uint32_t* heads;  // TLSF list heads (2,048 words, LDS)
};

constexpr int kOrdDir = 2;                          // directory registers
constexpr uint32_t kOrdSlots = 64u * kOrdDir;      // chunk slots per table
constexpr uint32_t kOrdMaxFree = 32u * kOrdSlots;  // free blocks always held
constexpr uint32_t kOrdTlsfHeadBytes = kTlsfClasses * 4u;

// Bytes of chunk slots of the address table (a) and of best fit's key
// table (b) for an algorithm.
__host__ __device__ constexpr uint32_t ord_chunk_a(int algo) {
  return 64u * (seg_like(algo) ? 16u : 8u);
}
__host__ __device__ constexpr uint32_t ord_chunk_b(int algo) {
  return algo == kBestFit ? 64u * 8u : 0u;
}
// Device bytes per wave: every slot of both tables and every live entry
// (slots and entries held in LDS keep an unused place here).
// The address table of segregated fit (1 KiB a chunk) is the largest; best
// fit's two tables of 512 B chunks take as much together.
constexpr uint64_t kOrdTableBytes = (uint64_t)kOrdSlots * (64u * 16u);
__host__ __device__ constexpr uint64_t ord_dev_bytes(uint32_t cap_live) {
  return kOrdTableBytes + (uint64_t)cap_live * 8u;
}

// Split a wave's pool (`pool` bytes, of which `slot_bytes` are meant for
// chunk slots) and its device slot for an algorithm.
__device__ __forceinline__ OrdMem ord_mem(int algo, HDA_LDS uint8_t* pool, uint32_t pool_bytes,
                                          uint32_t slot_bytes, HDA_GLOBAL uint8_t* dev,
                                          uint32_t cap_live) {
  OrdMem m;
  uint32_t off = 0;
  m.heads = (HDA_LDS uint32_t*)pool;
  if (algo == kTlsf) off += kOrdTlsfHeadBytes;
  const uint32_t ca = ord_chunk_a(algo), cb = ord_chunk_b(algo);
  uint32_t na = slot_bytes / (ca + cb);
  na = na < kOrdSlots ? na : kOrdSlots;
  const uint32_t room = pool_bytes > off ? pool_bytes - off : 0u;
  na = na * (ca + cb) <= room ? na : room / (ca + cb);
  m.ta_l = pool + off;
  m.ta_n = na;
  off += na * ca;
  m.tb_l = pool + off;
  m.tb_n = cb ? na : 0u;
  off += cb ? na * cb : 0u;
  m.ta_g = dev;
  m.tb_g = dev + (uint64_t)kOrdSlots * ca;
  m.ll = (HDA_LDS Ent*)(pool + off);
  const uint32_t nl = pool_bytes > off ? (pool_bytes - off) / 8u : 0u;
  m.ll_n = nl < cap_live ? nl : cap_live;
  m.gl = (HDA_GLOBAL Ent*)(dev + kOrdTableBytes);
  return m;
}

template <int ALGO>
struct OrdHeap {
  static constexpr int D = kOrdDir;
  static constexpr bool kSeg = ALGO == kSegFit || ALGO == kTlsf;
  static constexpr bool kKeys = ALGO == kBestFit;
  static constexpr bool kMax = ALGO == kFirstFit || ALGO == kNextFit;
  using TA = Hal<kSeg, false, kMax, D>;
  using TB = Hal<false, true, false, D>;
  using Row = typename TA::Row;

  TA ta;
  TB tb;
  OrdMem m;
  int64_t arena;
  uint32_t shift, ag;
  uint32_t F, L, rover;
  uint32_t capF, capL;
  uint32_t hd;      // segregated fit: lane k = head of class k's list (kNone: empty)
  uint64_t bm;      // segregated fit: class bitmap; TLSF: first-level bitmap
  uint32_t slb;     // TLSF: lane fl = bitmap of the 32 sub-classes of level fl

  __device__ __forceinline__ OrdHeap(const OrdMem& mem, const HeapRegs& h, uint32_t cap_free,
                                     uint32_t cap_live)
      : m(mem), arena(h.arena), shift(h.shift), ag(h.ag),
        capF(cap_free < kOrdMaxFree ? cap_free : kOrdMaxFree), capL(cap_live) {}

  // ---- live table ----
  __device__ __forceinline__ Ent lget(uint32_t i) const {
    wave_sync();
    if (i < m.ll_n) return m.ll[i];
    return m.gl[i];
  }
  __device__ __forceinline__ void lset(uint32_t i, Ent e) const {
    wave_sync();
    if (i < m.ll_n) m.ll[i] = e; else m.gl[i] = e;  // every lane, same value
  }
  __device__ __forceinline__ Ent lchunk(uint32_t base) const {  // base: multiple of 64
    wave_sync();
    const uint32_t i = base + lane_id();
    if (base < m.ll_n) return m.ll[i];
    return m.gl[i];
  }

  // ---- class lists (segregated fit, TLSF) ----
  __device__ __forceinline__ uint32_t cls(uint32_t sg) const {
    return ALGO == kTlsf ? tlsf_class(sg, shift) : floor_log2_u32(sg) + shift;
  }
  __device__ __forceinline__ uint32_t head(uint32_t c) const {
    if constexpr (ALGO == kTlsf) {
      wave_sync();
      return m.heads[c];
    } else {
      return rdlane(hd, c);
    }
  }
  __device__ __forceinline__ void set_head(uint32_t c, uint32_t a) {
    if constexpr (ALGO == kTlsf) {
      wave_sync();
      m.heads[c] = a;
    } else {
      hd = put_lane(hd, c, a);
    }
  }
  __device__ __forceinline__ void bit_set(uint32_t c) {
    if constexpr (ALGO == kTlsf) {
      slb = put_lane(slb, c >> 5, rdlane(slb, c >> 5) | (1u << (c & 31u)));
      bm |= 1ull << (c >> 5);
    } else {
      bm |= 1ull << c;
    }
  }
  __device__ __forceinline__ void bit_clear(uint32_t c) {
    if constexpr (ALGO == kTlsf) {
      const uint32_t w = rdlane(slb, c >> 5) & ~(1u << (c & 31u));
      slb = put_lane(slb, c >> 5, w);
      bm &= w == 0u ? ~(1ull << (c >> 5)) : ~0ull;
    } else {
      bm &= ~(1ull << c);
    }
  }
  // field f (2 next, 3 prev) of the free block at address a
  __device__ __forceinline__ void set_link(uint32_t a, uint32_t f, uint32_t x) {
    uint32_t ci, p;
    Row r;
    ta.locate(0u, a, ci, r, p);
    ta.store_field(ta.slot(ci), p, f, x);
  }
  // Unlink block (a, s) with links (nx, pv) from its class list.
  __device__ __forceinline__ void unlink(uint32_t s, uint32_t nx, uint32_t pv) {
    const uint32_t c = cls(s);
    if (pv == kNone) {
      set_head(c, nx);
      if (nx == kNone) bit_clear(c);
    } else {
      set_link(pv, 2u, nx);
    }
    if (nx != kNone) set_link(nx, 3u, pv);
  }
  // Make block (a, s) the head of its class list (Alg. 4-5 push); returns
  // the old head, the block's next link.
  __device__ __forceinline__ uint32_t push(uint32_t a, uint32_t s) {
    const uint32_t c = cls(s);
    const uint32_t oh = head(c);
    if (oh != kNone) set_link(oh, 3u, a);
    set_head(c, a);
    bit_set(c);
    return oh;
  }

  // Alg. 6: one free block [0, A).
  __device__ __forceinline__ void init() {
    ta.init(m.ta_l, m.ta_g, m.ta_n);
    F = 1; L = 0; rover = 0;
    hd = kNone; bm = 0ull; slb = 0u;
    if constexpr (ALGO == kTlsf) {
      for (uint32_t c = 0; c < kTlsfClasses; c += 64u) {
        wave_sync();
        m.heads[c + lane_id()] = kNone;
      }
    }
    if constexpr (kSeg) {
      const uint32_t c = cls(ag);
      set_head(c, 0u);
      bit_set(c);
    }
    ta.start(0u, ag, kNone, kNone);
    if constexpr (kKeys) {
      tb.init(m.tb_l, m.tb_g, m.tb_n);
      tb.start(0u, ag, kNone, kNone);
    }
  }

  // Commit an allocation of sg granules from block (a, s) at position p of
  // chunk ci of the address table (row r just loaded); Alg. 1 / Alg. 4: the
  // block is cut from the low end.
  __device__ __forceinline__ int64_t commit(uint32_t ci, uint32_t p, const Row& r, uint32_t a,
                                            uint32_t s, uint32_t sg) {
    if (s > sg) {
      const uint32_t sl = ta.slot(ci);
      ta.store_entry(sl, p, a + sg, s - sg, kNone, kNone);
      if (p == 0u) dir_put(ta.dk0, ci, a + sg);
      if (kMax) {
        const Row o = TA::pick(lane_id() == p, Row{a + sg, s - sg, kNone, kNone}, r);
        dir_put(ta.dmx, ci, wave_max(o.s));
      }
    } else {
      ta.erase_at(ci, p, r);
      --F;
    }
    lset(L, mk_ent(a, sg));
    ++L;
    if (ALGO == kNextFit) rover = a + sg;
    return (int64_t)((uint64_t)a << shift);
  }

  // Allocate sg granules; kreq is the request's byte class (segregated fit)
  // or request class (TLSF).  Returns the byte offset, -1 or kENoMeta.
  __device__ __forceinline__ int64_t alloc(uint32_t sg, uint32_t kreq) {
    const uint32_t lane = lane_id();
    if constexpr (ALGO == kFirstFit) {
      const uint32_t ci = ta.first_fit_chunk(sg, 0u);
      if (ci == kNone) return kFail;
      const Row r = ta.load(ta.slot(ci));
      const uint32_t p = ctz64(ballot(r.s >= sg));
      const uint32_t a = rdlane(r.a, p), s = rdlane(r.s, p);
      if (L >= capL) return kENoMeta;
      return commit(ci, p, r, a, s, sg);
    } else if constexpr (ALGO == kNextFit) {
      // the search starts at the first block whose end lies past the rover:
      // the last block starting at or below it, if it reaches past it, else
      // the block after that one (R9-R11); then cyclically
      uint32_t ci0, p0;
      Row r0;
      ta.locate(0u, rover, ci0, r0, p0);
      uint32_t ci = kNone, p = 0;
      Row r;
      if (ci0 != kNone) {
        const uint32_t n = ta.count(ci0);
        const uint64_t past = ballot(lane < n && r0.a + r0.s > rover);
        // past != 0: its lowest lane is the start; else the start is the
        // first entry of the next chunk
        const uint32_t st = past != 0ull ? ctz64(past) : 64u;
        const uint64_t fit = ballot(lane < n && lane >= st && r0.s >= sg);
        if (fit != 0ull) {
          ci = ci0; p = ctz64(fit); r = r0;
        } else {
          const uint32_t c1 = ta.first_fit_chunk(sg, ci0 + 1u);
          const uint32_t c2 = c1 != kNone ? c1 : ta.first_fit_chunk(sg, 0u);
          if (c2 == kNone) return kFail;
          ci = c2;
          r = c2 == ci0 ? r0 : ta.load(ta.slot(c2));
          p = ctz64(ballot(lane < ta.count(c2) && r.s >= sg));
        }
      } else {
        const uint32_t c2 = ta.first_fit_chunk(sg, 0u);
        if (c2 == kNone) return kFail;
        ci = c2;
        r = ta.load(ta.slot(c2));
        p = ctz64(ballot(lane < ta.count(c2) && r.s >= sg));
      }
      const uint32_t a = rdlane(r.a, p), s = rdlane(r.s, p);
      if (L >= capL) return kENoMeta;
      return commit(ci, p, r, a, s, sg);
    } else if constexpr (ALGO == kBestFit) {
      // smallest key (size, address) at or above (sg, 0)
      uint32_t ci, p;
      typename TB::Row r;
      tb.insert_pos(sg, 0u, ci, r, p);
      if (p >= tb.count(ci)) {
        if (ci + 1u >= tb.nc) return kFail;
        ci = ci + 1u;
        r = tb.load(tb.slot(ci));
        p = 0u;
      }
      const uint32_t s = rdlane(r.s, p), a = rdlane(r.a, p);
      if (s < sg) return kFail;  // (only an empty heap's sentinel-free chunk)
      if (L >= capL) return kENoMeta;
      tb.erase_at(ci, p, r);
      if (s > sg) tb.insert_key(a + sg, s - sg);
      uint32_t cj, q;
      Row ra;
      ta.locate(0u, a, cj, ra, q);
      return commit(cj, q, ra, a, s, sg);
    } else {
      // class of the first non-empty list at or above the request's
      uint32_t c;
      if constexpr (ALGO == kTlsf) {
        if (kreq >= kTlsfClasses) return kFail;
        const uint32_t fl = kreq >> 5, sl = kreq & 31u;
        const uint32_t m2 = rdlane(slb, fl) & (~0u << sl);
        if (m2 != 0u) {
          c = (fl << 5) | (uint32_t)__builtin_ctz(m2);
        } else {
          const uint64_t m1 = fl < 63u ? bm & (~0ull << (fl + 1u)) : 0ull;
          if (m1 == 0ull) return kFail;
          const uint32_t f2 = ctz64(m1);
          c = (f2 << 5) | (uint32_t)__builtin_ctz(rdlane(slb, f2));
        }
      } else {
        if (kreq >= 64u) return kFail;
        const uint64_t mk = bm & (~0ull << kreq);
        if (mk == 0ull) return kFail;
        c = ctz64(mk);
      }
      const uint32_t a = head(c);
      uint32_t ci, p;
      Row r;
      ta.locate(0u, a, ci, r, p);
      const uint32_t s = rdlane(r.s, p), nx = rdlane(r.nx, p);
      if (L >= capL) return kENoMeta;
      // pop the head (Alg. 4), keeping the lists' invariants (R20)
      set_head(c, nx);
      if (nx == kNone) bit_clear(c); else set_link(nx, 3u, kNone);
      if (s > sg) {
        // the remainder is pushed at the head of its class (Alg. 4)
        const uint32_t oh = push(a + sg, s - sg);
        ta.store_entry(ta.slot(ci), p, a + sg, s - sg, oh, kNone);
        if (p == 0u) dir_put(ta.dk0, ci, a + sg);
      } else {
        const Row rr = ta.load(ta.slot(ci));  // the links above may have changed it
        ta.erase_at(ci, p, rr);
        --F;
      }
      lset(L, mk_ent(a, sg));
      ++L;
      return (int64_t)((uint64_t)a << shift);
    }
  }

  // Release [x, x + sz) into the free blocks, merging with free neighbours
  // (Alg. 2 / Alg. 5).  Returns false, changing nothing, when a new free
  // entry would exceed the capacity.
  __device__ __forceinline__ bool release(uint32_t x, uint32_t sz) {
    const uint32_t lane = lane_id();
    // the last free block below x and the one after it
    uint32_t ci, p;
    Row r;
    ta.locate(0u, x, ci, r, p);
    bool hasL = false, hasR = false;
    uint32_t la = 0, ls = 0, lnx = kNone, lpv = kNone;
    uint32_t ra = 0, rs = 0, rnx = kNone, rpv = kNone;
    uint32_t rci = 0, rp = 0;   // position of the block after x
    if (ci != kNone) {
      la = rdlane(r.a, p); ls = rdlane(r.s, p);
      if (kSeg) { lnx = rdlane(r.nx, p); lpv = rdlane(r.pv, p); }
      hasL = la + ls == x;
      if (p + 1u < ta.count(ci)) {
        rci = ci; rp = p + 1u;
        ra = rdlane(r.a, rp); rs = rdlane(r.s, rp);
        if (kSeg) { rnx = rdlane(r.nx, rp); rpv = rdlane(r.pv, rp); }
        hasR = ra == x + sz;
      } else if (ci + 1u < ta.nc && dir_get(ta.dk0, ci + 1u) == x + sz) {
        rci = ci + 1u; rp = 0u;
        const Row r2 = ta.load(ta.slot(rci));
        ra = rdlane(r2.a, 0u); rs = rdlane(r2.s, 0u);
        if (kSeg) { rnx = rdlane(r2.nx, 0u); rpv = rdlane(r2.pv, 0u); }
        hasR = true;
      }
    } else if (ta.nc != 0u && ta.count(0u) != 0u && dir_get(ta.dk0, 0u) == x + sz) {
      rci = 0u; rp = 0u;
      const Row r2 = ta.load(ta.slot(0u));
      ra = rdlane(r2.a, 0u); rs = rdlane(r2.s, 0u);
      if (kSeg) { rnx = rdlane(r2.nx, 0u); rpv = rdlane(r2.pv, 0u); }
      hasR = true;
    }
    if (!hasL && !hasR && F >= capF) return false;
    const uint32_t ma = hasL ? la : x;
    const uint32_t ms = (hasL ? ls : 0u) + sz + (hasR ? rs : 0u);
    uint32_t nx = kNone;
    if constexpr (kSeg) {
      // unlink the free neighbours, then push the merged block (R21)
      if (hasL) {
        unlink(ls, lnx, lpv);
        // unlinking the left block rewrote the links of its list
        // neighbours, which may include the right block
        rpv = rpv == la ? lpv : rpv;
        rnx = rnx == la ? lnx : rnx;
      }
      if (hasR) unlink(rs, rnx, rpv);
      nx = push(ma, ms);
    }
    if constexpr (kKeys) {
      if (hasL) tb.erase_key(la, ls);
      if (hasR) tb.erase_key(ra, rs);
      tb.insert_key(ma, ms);
    }
    if (hasL) {
      ta.store_entry(ta.slot(ci), p, ma, ms, nx, kNone);
      if (kMax) {
        const Row o = TA::pick(lane == p, Row{ma, ms, kNone, kNone}, r);
        dir_put(ta.dmx, ci, wave_max(o.s));
      }
      if (hasR) {
        // the block after x: at rci / rp, still (entries were rewritten in
        // place only)
        const Row rr = ta.load(ta.slot(rci));
        ta.erase_at(rci, rp, rr);
        --F;
      }
    } else if (hasR) {
      ta.store_entry(ta.slot(rci), rp, ma, ms, nx, kNone);
      if (rp == 0u) dir_put(ta.dk0, rci, ma);
      if (kMax) dir_put(ta.dmx, rci, wave_max(ta.load(ta.slot(rci)).s));
    } else {
      uint32_t ic, ip;
      Row ir;
      ta.insert_pos(0u, x, ic, ir, ip);
      Row e = TA::sentinel();
      e.a = x; e.s = sz; e.nx = nx; e.pv = kNone;
      ta.insert_at(ic, ip, ir, e);
      ++F;
    }
    return true;
  }

  // Free live entry idx except its first floor(cut * size / 2^31) granules
  // (partial deallocation, sequential fits; cut < 2^31).  Returns the byte
  // offset of the released part or kENoMeta.
  __device__ __forceinline__ int64_t free_index(uint32_t idx, uint32_t cut) {
    const Ent v = lget(idx);
    const uint32_t bx = ent_a(v), bsz = ent_s(v);
    const uint32_t t = (kSeg || cut == 0u) ? 0u : (uint32_t)(((uint64_t)cut * bsz) >> 31);
    const uint32_t x = bx + t, sz = bsz - t;
    if (!release(x, sz)) return kENoMeta;
    if (t != 0u) {
      lset(idx, mk_ent(bx, t));
    } else {
      const uint32_t last = L - 1u;
      const Ent e = lget(last);
      lset(idx, e);
      L = last;
    }
    return (int64_t)((uint64_t)x << shift);
  }

  __device__ __forceinline__ int64_t free_draw(uint32_t r, uint32_t cut) {
    if (L == 0u) return kFail;
    return free_index((uint32_t)(((uint64_t)r * (uint64_t)L) >> 32), cut);
  }

  // Canonical state (format in hda.h).
  __device__ __forceinline__ int64_t dump(int64_t* out, int64_t cap) {
    const uint32_t lane = lane_id();
    const int64_t lists = ALGO == kTlsf ? kTlsfClasses : (ALGO == kSegFit ? 64 : 0);
    const int64_t need = 4 + 2 * (int64_t)F + 2 * (int64_t)L + (kSeg ? lists + (int64_t)F : 0);
    if (out == nullptr || need > cap) return need;
    const uint32_t sh = shift;
    wave_sync();
    if (lane == 0) out[0] = F;
    int64_t* fo = out + 1;
    uint32_t k = 0;
    for (uint32_t ci = 0; ci < ta.nc; ++ci) {
      const Row r = ta.load(ta.slot(ci));
      const uint32_t n = ta.count(ci);
      wave_sync();
      if (lane < n) {
        fo[2 * (k + lane)] = (int64_t)((uint64_t)r.a << sh);
        fo[2 * (k + lane) + 1] = (int64_t)((uint64_t)r.s << sh);
      }
      k += n;
    }
    int64_t* lo = out + 1 + 2 * (int64_t)F;
    wave_sync();
    if (lane == 0) lo[0] = L;
    for (uint32_t base = 0; base < L; base += 64u) {
      const Ent e = lchunk(base);
      const uint32_t i = base + lane;
      wave_sync();
      if (i < L) {
        lo[1 + 2 * i] = (int64_t)((uint64_t)ent_a(e) << sh);
        lo[2 + 2 * i] = (int64_t)((uint64_t)ent_s(e) << sh);
      }
    }
    int64_t* tail = lo + 1 + 2 * (int64_t)L;
    wave_sync();
    if (lane == 0) {
      tail[0] = ALGO == kNextFit ? (int64_t)((uint64_t)rover << sh) : -1;
      tail[1] = kSeg ? (int64_t)bm : 0;
    }
    if constexpr (kSeg) {
      // each class: its length, then its blocks from the head along the
      // next links
      int64_t* ls = tail + 2;
      uint32_t pos = 0;
      for (uint32_t c = 0; c < (uint32_t)lists; ++c) {
        bool nonempty;
        if constexpr (ALGO == kTlsf) nonempty = (rdlane(slb, c >> 5) >> (c & 31u)) & 1u;
        else nonempty = (bm >> c) & 1ull;
        uint32_t n = 0;
        if (nonempty) {
          uint32_t a = head(c);
          // (bounded by the section's words even if a list were corrupt)
          while (a != kNone && pos + 1u + n < (uint32_t)lists + F) {
            wave_sync();
            if (lane == 0) ls[pos + 1u + n] = (int64_t)((uint64_t)a << sh);
            uint32_t ci, p;
            Row r;
            ta.locate(0u, a, ci, r, p);
            a = rdlane(r.nx, p);
            ++n;
          }
        }
        wave_sync();
        if (lane == 0) ls[pos] = n;
        pos += 1u + n;
      }
    }
    return need;
  }
};

}  // namespace hda
