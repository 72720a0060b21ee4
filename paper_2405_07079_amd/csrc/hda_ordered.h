// Ordered replay core: one wavefront replays one heap with its free blocks
// kept in address order, so that every step of Alg. 1-5 costs a fixed number
// of wave operations however many free blocks the heap has.
//
// Free blocks form a sorted array of 64-entry chunks, one entry per lane --
// the hybrid array list of App. A, whose traversal costs O(n/m + m) on one
// CPU thread.  Here a directory held in D VGPRs replaces the walk over the
// chunk list: lane l of directory register v describes chunk 64 v + l in
// order (its storage slot, its number of entries, its first key and, for
// first and next fit, the largest block in it).  Finding the chunk that
// holds a key, or the first chunk holding a block of at least s granules,
// is one ballot per directory register; finding the entry inside it is one
// chunk load and one ballot.  A full chunk splits into 33 + 32 entries; a
// chunk that drops below 32 entries merges with a neighbour or takes entries
// from it.  So while there are two or more chunks each holds at least 32
// entries, and the directory's 64 D chunks always hold 2,048 D free blocks.
//
// A free block's entry is keyed by its END granule address.  Free blocks do
// not overlap, so this is also address order, and Alg. 1 / Alg. 4 cut an
// allocation from the low end of a block: the remainder keeps its end, so
// splitting a block rewrites its size (or its record) and never its place.
// The block ending at a freed block's start is an exact key match; the one
// after it is the next entry.
//
// Per algorithm:
//  * first fit (Sec. II-A): entries (end, size); the first chunk whose
//    largest block fits, then the first fitting entry in it.
//  * next fit (Sec. II-A, Sec. IV): the first block ending past the rover
//    is located like a key; the search runs on from there through the
//    directory and wraps once.
//  * best fit (Alg. 3): entries (end, size) and a second sorted chunk table
//    of keys (size, end) -- among blocks of one size the lowest end is the
//    lowest address; the smallest key at or above (s, 0) is the best fit.
//  * segregated fit (Alg. 4-5) and TLSF (Sec. V-B): entries (end, record).
//    A record holds the block's address and size and its class-list links
//    (next and previous record, NIL = kNone), as Alg. 4-5 keep them; record
//    numbers never change while a block is free, so unlinking and pushing
//    are stores with no search.  Free record numbers are bits of a VGPR
//    pair (lane l: records 64 l .. 64 l + 63).  List heads are in a VGPR
//    (segregated fit: lane k heads class k) or in LDS (TLSF's 2,048
//    classes); the bitmaps are a scalar (segregated fit; TLSF's first level)
//    and a VGPR (TLSF's second level: lane fl holds level fl's 32 bits).
//    The paper's address-keyed hash lookup ht[addr] becomes the key lookup
//    in the table.
//
// Results equal those of the other cores and the oracle: selection,
// splitting, merging and the class lists follow the same definitions.
//
// Storage: chunk slots, records and live entries below the LDS counts given
// at construction are in the wave's LDS pool, the rest in its device-memory
// slot.  Every memory access is preceded by wave_sync() (a no-op on the GPU;
// the CPU wave emulation switches lanes there).  As in the other cores,
// values that feed a cross-lane operation are never produced under a
// lane-dependent branch, and every single-entry write is done by all lanes
// with the same value.
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

// The lanes below n as a mask (n <= 64 or more): lane conditions of a ballot
// are applied on the scalar side instead of being combined per lane.
__device__ __forceinline__ uint64_t lanes_below(uint32_t n) {
  return n >= 64u ? ~0ull : (1ull << n) - 1ull;
}

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
    const uint32_t moved = wave_shr1(carry, v[k]);  // lane 0 takes the carry
    const uint32_t g = 64u * (uint32_t)k + lane;
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
    const uint32_t moved = wave_shl1(next0, v[k]);  // lane 63 takes the next register's lane 0
    const uint32_t g = 64u * (uint32_t)k + lane;
    v[k] = g >= i ? moved : v[k];
  }
}

// One table of sorted chunks of 8-byte entries (key, value): the key is a
// block's end granule, the value its size or its record.  KEY64: sorted by
// (value, key) instead (best fit's (size, end) keys).  MAXS: the directory
// keeps each chunk's largest value (first and next fit: the largest size).
template <bool KEY64, bool MAXS, int D>
struct Hal {
  static constexpr uint32_t NC = 64u * D;  // chunk slots
  static constexpr uint32_t CB = 64u * 8u; // bytes per chunk

  // this lane's entry of a loaded chunk; positions past the chunk's count
  // hold the sentinel (key kNone, value 0, or value kNone when sorted by
  // value), which sorts after every real entry and fits no request
  struct Row {
    uint32_t a, s;
  };

  static constexpr int ND = D;
  HDA_LDS uint8_t* lb;     // slots [0, nl) in LDS
  HDA_GLOBAL uint8_t* gb;  // slot i >= nl at gb + i * CB in device memory
  uint32_t nl, nl_req;     // LDS slots (nl_req as asked for, nl within NC)
  uint32_t dsl[D], dct[D], dk0[D], dk1[D], dmx[D];  // slot, count, first key, max value
  uint64_t used[D];                                 // slots in use
  uint32_t nc;                                      // chunks

  static constexpr uint32_t kSentS = KEY64 ? kNone : 0u;

  __device__ __forceinline__ static Row sentinel() { return Row{kNone, kSentS}; }

  __device__ __forceinline__ void init(HDA_LDS uint8_t* l, HDA_GLOBAL uint8_t* g, uint32_t n_lds) {
    lb = l;
    gb = g;
    nl_req = n_lds;
    nl = n_lds < NC ? n_lds : NC;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      dsl[k] = 0u; dct[k] = 0u; dk0[k] = kNone; dk1[k] = kNone; dmx[k] = 0u;
      used[k] = 0ull;
    }
    nc = 0;
  }

  // ---- chunk memory (slot ids are below NC; the clamps keep every access
  // inside the table whatever happens) ----
  __device__ __forceinline__ Row load(uint32_t sl) const {
    wave_sync();
    sl = sl < NC ? sl : NC - 1u;
    const uint32_t lane = lane_id();
    u32x2 v;
    if (sl < nl) {
      v = *(const HDA_LDS u32x2*)(lb + sl * CB + lane * 8u);
    } else {
      v = *(const HDA_GLOBAL u32x2*)(gb + (uint64_t)sl * CB + lane * 8u);
      settle(v[0]);
      settle(v[1]);
    }
    return Row{v[0], v[1]};
  }
  __device__ __forceinline__ void store(uint32_t sl, const Row& r) const {
    wave_sync();
    sl = sl < NC ? sl : NC - 1u;
    const uint32_t lane = lane_id();
    u32x2 v;
    v[0] = r.a; v[1] = r.s;
    if (sl < nl) *(HDA_LDS u32x2*)(lb + sl * CB + lane * 8u) = v;
    else *(HDA_GLOBAL u32x2*)(gb + (uint64_t)sl * CB + lane * 8u) = v;
  }
  // field f (0 key, 1 value) of entry p, written by every lane
  __device__ __forceinline__ void store_field(uint32_t sl, uint32_t p, uint32_t f,
                                              uint32_t x) const {
    wave_sync();
    sl = sl < NC ? sl : NC - 1u;
    const uint32_t off = (p & 63u) * 8u + (f & 1u) * 4u;
    if (sl < nl) *(HDA_LDS uint32_t*)(lb + sl * CB + off) = x;
    else *(HDA_GLOBAL uint32_t*)(gb + (uint64_t)sl * CB + off) = x;
  }
  __device__ __forceinline__ void store_entry(uint32_t sl, uint32_t p, uint32_t a,
                                              uint32_t s) const {
    wave_sync();
    sl = sl < NC ? sl : NC - 1u;
    u32x2 v;
    v[0] = a; v[1] = s;
    const uint32_t off = (p & 63u) * 8u;
    if (sl < nl) *(HDA_LDS u32x2*)(lb + sl * CB + off) = v;
    else *(HDA_GLOBAL u32x2*)(gb + (uint64_t)sl * CB + off) = v;
  }

  // ---- keys ----
  // Lanes whose key (r1, r0) is <= (k1, k0) (strict: <); keyed by r0 alone
  // unless KEY64.  Each comparison is one ballot; they are combined on the
  // scalar side.
  __device__ __forceinline__ static uint64_t key_ballot(uint32_t r1, uint32_t r0, uint32_t k1,
                                                        uint32_t k0, bool strict) {
    if constexpr (!KEY64) return strict ? ballot(r0 < k0) : ballot(r0 <= k0);
    // (r1, r0) as one 64-bit value: one vector compare
    const uint64_t r = ((uint64_t)r1 << 32) | r0, k = ((uint64_t)k1 << 32) | k0;
    return strict ? ballot(r < k) : ballot(r <= k);
  }
  // chunks whose first key is <= (k1, k0) (strict: <)
  __device__ __forceinline__ uint32_t count_first(uint32_t k1, uint32_t k0, bool strict) const {
    uint32_t n = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const uint32_t base = 64u * (uint32_t)k;
      const uint64_t le = key_ballot(dk1[k], dk0[k], k1, k0, strict);
      n += (uint32_t)__builtin_popcountll(le & lanes_below(nc > base ? nc - base : 0u));
    }
    return n;
  }

  __device__ __forceinline__ uint32_t slot(uint32_t ci) const { return dir_get(dsl, ci); }
  __device__ __forceinline__ uint32_t count(uint32_t ci) const { return dir_get(dct, ci); }

  // Directory entry of chunk ci from its row (n entries).
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
  __device__ __forceinline__ void start(uint32_t a, uint32_t s) {
    const uint32_t sl = take_slot();
    Row r = sentinel();
    const bool me = lane_id() == 0u;
    r.a = me ? a : r.a;
    r.s = me ? s : r.s;
    store(sl, r);
    nc = 1;
    dir_put(dsl, 0u, sl);
    describe(0u, r, 1u);
  }

  // Row shifted: lane l receives lane src(l) of r (the sentinel when !ok).
  __device__ __forceinline__ static Row pull(const Row& r, uint32_t src, bool ok) {
    const uint32_t s = src & 63u;
    Row o{shfl(r.a, s), shfl(r.s, s)};
    o.a = ok ? o.a : kNone;
    o.s = ok ? o.s : kSentS;
    return o;
  }
  __device__ __forceinline__ static Row pick(bool c, const Row& x, const Row& y) {
    return Row{c ? x.a : y.a, c ? x.s : y.s};
  }
  // r with lane p's entry replaced
  __device__ __forceinline__ static Row with(const Row& r, uint32_t p, uint32_t a, uint32_t s) {
    const bool me = lane_id() == p;
    return Row{me ? a : r.a, me ? s : r.s};
  }

  // Insert entry e at position p (0 <= p <= count) of chunk ci, whose row r
  // is current.  The caller guarantees order and capacity.
  __device__ __forceinline__ void insert_at(uint32_t ci, uint32_t p, const Row& r, const Row& e) {
    const uint32_t lane = lane_id();
    const uint32_t n = count(ci), sl = slot(ci);
    // the row moved up one lane (lane 0: the sentinel)
    const Row up{wave_shr1(kNone, r.a), wave_shr1(kSentS, r.s)};
    if (n < 64u) {
      const Row o = pick(lane < p, r, pick(lane == p, e, up));
      store(sl, o);
      describe(ci, o, n + 1u);
      return;
    }
    // split: the 65 entries c[0..64] become 33 here and 32 in a new chunk
    // after it; c[i] = r[i] (i < p), e (i == p), r[i - 1] (i > p)
    const uint32_t ns = take_slot();
    Row left = pick(lane < p, r, pick(lane == p, e, up));
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

  // Remove the entry at position p of chunk ci (row r current), then keep
  // every chunk at 32 entries or more while there are two or more.
  __device__ __forceinline__ void erase_at(uint32_t ci, uint32_t p, const Row& r) {
    const uint32_t lane = lane_id();
    const uint32_t n = count(ci) - 1u, sl = slot(ci);
    // the row moved down one lane (lane 63: the sentinel)
    const Row down{wave_shl1(kNone, r.a), wave_shl1(kSentS, r.s)};
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

  // The last chunk whose first key is <= (k1, k0): ci (kNone if every chunk
  // starts above it), its row, and p = the position of the last entry <= the
  // key in it.
  __device__ __forceinline__ void locate(uint32_t k1, uint32_t k0, uint32_t& ci, Row& r,
                                         uint32_t& p) const {
    const uint32_t c = count_first(k1, k0, false);
    if (c == 0u) { ci = kNone; p = kNone; return; }
    ci = c - 1u;
    r = load(slot(ci));
    const uint32_t n = count(ci);
    p = (uint32_t)__builtin_popcountll(key_ballot(r.s, r.a, k1, k0, false) & lanes_below(n)) - 1u;
  }
  // Where a new key goes: chunk ci (the last one starting below it, else
  // the first), its row, and the position of the first entry above it.
  __device__ __forceinline__ void insert_pos(uint32_t k1, uint32_t k0, uint32_t& ci, Row& r,
                                             uint32_t& p) const {
    const uint32_t c = count_first(k1, k0, true);
    ci = c == 0u ? 0u : c - 1u;
    r = load(slot(ci));
    const uint32_t n = count(ci);
    p = (uint32_t)__builtin_popcountll(key_ballot(r.s, r.a, k1, k0, true) & lanes_below(n));
  }
  // (value, key) tables: insert and remove one key
  __device__ __forceinline__ void insert_key(uint32_t a, uint32_t s) {
    uint32_t ci, p;
    Row r;
    insert_pos(s, a, ci, r, p);
    insert_at(ci, p, r, Row{a, s});
  }
  __device__ __forceinline__ void erase_key(uint32_t a, uint32_t s) {
    uint32_t ci, p;
    Row r;
    locate(s, a, ci, r, p);
    erase_at(ci, p, r);
  }
  // first chunk at or after `from` whose largest value is >= sg (MAXS
  // tables), or kNone
  __device__ __forceinline__ uint32_t first_fit_chunk(uint32_t sg, uint32_t from) const {
    uint32_t c = kNone;
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
      const uint32_t base = 64u * (uint32_t)k;
      const uint64_t m = ballot(dmx[k] >= sg) & lanes_below(nc > base ? nc - base : 0u) &
                         ~lanes_below(from > base ? from - base : 0u);
      c = m != 0ull ? 64u * (uint32_t)k + ctz64(m) : c;
    }
    return c;
  }
};

// Where one heap's tables live.  Table slots, records and live entries below
// the LDS counts are in the wave's LDS pool; the others are in its device
// slot.
struct OrdMem {
  HDA_LDS uint8_t* ta_l;
  HDA_GLOBAL uint8_t* ta_g;
  uint32_t ta_n;
  HDA_LDS uint8_t* tb_l;     // best fit's key table
  HDA_GLOBAL uint8_t* tb_g;
  uint32_t tb_n;
  HDA_LDS u32x4* rec_l;      // segregated fit / TLSF records
  HDA_GLOBAL u32x4* rec_g;
  uint32_t rec_n;
  HDA_LDS Ent* ll;
  HDA_GLOBAL Ent* gl;
  uint32_t ll_n;
  HDA_LDS uint32_t* heads;   // TLSF list heads (2,048 words, LDS)
};

constexpr int kOrdDir = 2;                          // directory registers at most
constexpr uint32_t kOrdSlots = 64u * kOrdDir;      // chunk slots per table
constexpr uint32_t kOrdMaxFree = 32u * kOrdSlots;  // free blocks always held
constexpr uint32_t kOrdTlsfHeadBytes = kTlsfClasses * 4u;
constexpr uint32_t kOrdChunkBytes = 64u * 8u;
// Device bytes per wave: every chunk slot of the table (64 KiB), then best
// fit's key table or the records (64 KiB either), then the live table.
// Slots, records and entries held in LDS keep an unused place here.
constexpr uint64_t kOrdTableBytes = (uint64_t)kOrdSlots * kOrdChunkBytes;
constexpr uint64_t kOrdSecondBytes = (uint64_t)kOrdMaxFree * 16u;
static_assert(kOrdSecondBytes == kOrdTableBytes, "key table and records share one area");
__host__ __device__ constexpr uint64_t ord_dev_bytes(uint32_t cap_live) {
  return kOrdTableBytes + kOrdSecondBytes + (uint64_t)cap_live * 8u;
}

// Split a wave's pool (`pool_bytes`, of which `slot_bytes` are meant for the
// tables and records) and its device slot for an algorithm.
__device__ __forceinline__ OrdMem ord_mem(int algo, HDA_LDS uint8_t* pool, uint32_t pool_bytes,
                                          uint32_t slot_bytes, HDA_GLOBAL uint8_t* dev,
                                          uint32_t cap_live) {
  OrdMem m;
  uint32_t off = 0;
  m.heads = (HDA_LDS uint32_t*)pool;
  if (algo == kTlsf) off += kOrdTlsfHeadBytes;
  const uint32_t room = pool_bytes > off ? pool_bytes - off : 0u;
  const uint32_t area = slot_bytes < room ? slot_bytes : room;
  // first and next fit: every slot of the table; best fit: half for each of
  // its two tables; segregated fit, TLSF: half for table slots, half for
  // records
  const bool two = algo == kBestFit || seg_like(algo);
  uint32_t na = (two ? area / 2u : area) / kOrdChunkBytes;
  na = na < kOrdSlots ? na : kOrdSlots;
  m.ta_l = pool + off;
  m.ta_n = na;
  off += na * kOrdChunkBytes;
  m.tb_l = pool + off;
  m.tb_n = algo == kBestFit ? na : 0u;
  off += algo == kBestFit ? na * kOrdChunkBytes : 0u;
  uint32_t nr = seg_like(algo) ? (area / 2u) / 16u : 0u;
  nr = nr < kOrdMaxFree ? nr : kOrdMaxFree;
  m.rec_l = (HDA_LDS u32x4*)(pool + off);
  m.rec_n = nr;
  off += nr * 16u;
  m.ta_g = dev;
  m.tb_g = dev + kOrdTableBytes;
  m.rec_g = (HDA_GLOBAL u32x4*)(dev + kOrdTableBytes);
  m.ll = (HDA_LDS Ent*)(pool + off);
  const uint32_t nl = pool_bytes > off ? (pool_bytes - off) / 8u : 0u;
  m.ll_n = nl < cap_live ? nl : cap_live;
  m.gl = (HDA_GLOBAL Ent*)(dev + kOrdTableBytes + kOrdSecondBytes);
  return m;
}

// D: directory registers.  A heap starts with one; a request that finds a
// table at 64 chunks returns kOverflow before changing anything, and the
// heap continues with two (take()), which hold every table this core allows.
template <int ALGO, int D>
struct OrdHeap {
  static constexpr bool kSeg = ALGO == kSegFit || ALGO == kTlsf;
  static constexpr bool kKeys = ALGO == kBestFit;
  static constexpr bool kMax = ALGO == kFirstFit || ALGO == kNextFit;
  using TA = Hal<false, kMax, D>;
  using TB = Hal<true, false, D>;
  using Row = typename TA::Row;

  TA ta;
  TB tb;
  OrdMem m;
  int64_t arena;
  uint32_t shift, ag;
  uint32_t F, L, rover;
  uint32_t capF, capL;
  uint32_t hd;          // segregated fit: lane k = head record of class k (kNone: empty)
  uint64_t bm;          // segregated fit: class bitmap; TLSF: first-level bitmap
  uint32_t slb;         // TLSF: lane fl = bitmap of the 32 sub-classes of level fl
  uint32_t frl, frh;    // free records: lane l, bit b <=> record 64 l + b (low, high word)

  __device__ __forceinline__ OrdHeap(const OrdMem& mem, const HeapRegs& h, uint32_t cap_free,
                                     uint32_t cap_live)
      : m(mem), arena(h.arena), shift(h.shift), ag(h.ag),
        capF(cap_free < kOrdMaxFree ? cap_free : kOrdMaxFree), capL(cap_live) {}

  // ---- live table ----
  // (every lane reads the same entry; the halves are made wave-uniform so
  // that what is computed from them stays scalar)
  __device__ __forceinline__ Ent lget(uint32_t i) const {
    const Ent e = lraw(i);
    return mk_ent(uniform(ent_a(e)), uniform(ent_s(e)));
  }
  __device__ __forceinline__ Ent lraw(uint32_t i) const {
    wave_sync();
    if (i < m.ll_n) return m.ll[i];
    const Ent e = m.gl[i];
    settle((uint32_t)e);
    settle((uint32_t)(e >> 32));
    return e;
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

  // ---- records (segregated fit, TLSF): address, size, next, prev ----
  struct Rec {
    uint32_t a, s, nx, pv;
  };
  __device__ __forceinline__ u32x4 rec_raw(uint32_t i) const {
    wave_sync();
    i = i < kOrdMaxFree ? i : kOrdMaxFree - 1u;
    u32x4 v;
    if (i < m.rec_n) {
      v = m.rec_l[i];
    } else {
      v = m.rec_g[i];
      settle(v[0]); settle(v[1]); settle(v[2]); settle(v[3]);
    }
    return v;
  }
  __device__ __forceinline__ static Rec rec_of(const u32x4& v) {
    return Rec{uniform(v[0]), uniform(v[1]), uniform(v[2]), uniform(v[3])};
  }
  __device__ __forceinline__ Rec rec(uint32_t i) const { return rec_of(rec_raw(i)); }
  __device__ __forceinline__ void rec_put(uint32_t i, uint32_t a, uint32_t s, uint32_t nx,
                                          uint32_t pv) const {
    wave_sync();
    i = i < kOrdMaxFree ? i : kOrdMaxFree - 1u;
    u32x4 v;
    v[0] = a; v[1] = s; v[2] = nx; v[3] = pv;
    if (i < m.rec_n) m.rec_l[i] = v; else m.rec_g[i] = v;
  }
  // one field (2 next, 3 prev) of record i
  __device__ __forceinline__ void rec_link(uint32_t i, uint32_t f, uint32_t x) const {
    wave_sync();
    i = i < kOrdMaxFree ? i : kOrdMaxFree - 1u;
    if (i < m.rec_n) ((HDA_LDS uint32_t*)(m.rec_l + i))[f & 3u] = x;
    else ((HDA_GLOBAL uint32_t*)(m.rec_g + i))[f & 3u] = x;
  }
  __device__ __forceinline__ uint32_t rec_take() {
    const uint64_t m1 = ballot((frl | frh) != 0u);
    const uint32_t l = m1 != 0ull ? ctz64(m1) : 63u;
    const uint32_t wl = rdlane(frl, l), wh = rdlane(frh, l);
    const uint32_t b = wl != 0u ? (uint32_t)__builtin_ctz(wl)
                                : 32u + (uint32_t)__builtin_ctz(wh != 0u ? wh : 1u);
    const bool me = lane_id() == l;
    frl = me && b < 32u ? frl & ~(1u << b) : frl;
    frh = me && b >= 32u ? frh & ~(1u << (b - 32u)) : frh;
    return 64u * l + b;
  }
  __device__ __forceinline__ void rec_give(uint32_t i) {
    const bool me = lane_id() == (i >> 6);
    const uint32_t b = i & 63u;
    frl = me && b < 32u ? frl | (1u << b) : frl;
    frh = me && b >= 32u ? frh | (1u << (b - 32u)) : frh;
  }

  // ---- class lists (segregated fit, TLSF) ----
  __device__ __forceinline__ uint32_t cls(uint32_t sg) const {
    return ALGO == kTlsf ? tlsf_class(sg, shift) : floor_log2_u32(sg) + shift;
  }
  __device__ __forceinline__ uint32_t head(uint32_t c) const {
    if constexpr (ALGO == kTlsf) {
      wave_sync();
      return uniform(m.heads[c]);
    } else {
      return rdlane(hd, c);
    }
  }
  __device__ __forceinline__ void set_head(uint32_t c, uint32_t i) {
    if constexpr (ALGO == kTlsf) {
      wave_sync();
      m.heads[c] = i;
    } else {
      hd = put_lane(hd, c, i);
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
  // Unlink a block of sg granules with links (nx, pv) from its class list.
  __device__ __forceinline__ void unlink(uint32_t sg, uint32_t nx, uint32_t pv) {
    const uint32_t c = cls(sg);
    if (pv == kNone) {
      set_head(c, nx);
      if (nx == kNone) bit_clear(c);
    } else {
      rec_link(pv, 2u, nx);
    }
    if (nx != kNone) rec_link(nx, 3u, pv);
  }
  // Record i becomes the head of its class list (Alg. 4-5 push) with block
  // (a, sg).
  __device__ __forceinline__ void push(uint32_t i, uint32_t a, uint32_t sg) {
    const uint32_t c = cls(sg);
    const uint32_t oh = head(c);
    if (oh != kNone) rec_link(oh, 3u, i);
    rec_put(i, a, sg, oh, kNone);
    set_head(c, i);
    bit_set(c);
  }

  // Alg. 6: one free block [0, A).
  __device__ __forceinline__ void init() {
    ta.init(m.ta_l, m.ta_g, m.ta_n);
    F = 1; L = 0; rover = 0;
    hd = kNone; bm = 0ull; slb = 0u;
    if constexpr (kSeg) {
      // records 0 .. capF - 1 are free, then record 0 takes the arena
      const uint32_t base = 64u * lane_id();
      frl = base >= capF ? 0u : (capF - base >= 32u ? ~0u : (1u << (capF - base)) - 1u);
      frh = base + 32u >= capF ? 0u
            : (capF - base - 32u >= 32u ? ~0u : (1u << (capF - base - 32u)) - 1u);
      if constexpr (ALGO == kTlsf) {
        for (uint32_t c = 0; c < kTlsfClasses; c += 64u) {
          wave_sync();
          m.heads[c + lane_id()] = kNone;
        }
      }
      const uint32_t r0 = rec_take();
      push(r0, 0u, ag);
      ta.start(ag, r0);
    } else {
      frl = frh = 0u;
      ta.start(ag, ag);
    }
    if constexpr (kKeys) {
      tb.init(m.tb_l, m.tb_g, m.tb_n);
      tb.start(ag, ag);
    }
  }

  // First and next fit: the block at position p of chunk ci (row r current,
  // key e = its end, value s = its size) gives sg granules from its low end.
  __device__ __forceinline__ int64_t commit_fit(uint32_t ci, uint32_t p, const Row& r,
                                                uint32_t e, uint32_t s, uint32_t sg) {
    const uint32_t a = e - s;
    if (s > sg) {
      ta.store_field(ta.slot(ci), p, 1u, s - sg);  // the end stays
      if (kMax) dir_put(ta.dmx, ci, wave_max(TA::with(r, p, e, s - sg).s));
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
  __device__ __forceinline__ bool full_dir() const {
    return D < kOrdDir && (ta.nc >= 64u * D || (kKeys && tb.nc >= 64u * D));
  }

  // Continue a heap that ran with fewer directory registers: the same
  // chunks, records and live entries, the directories widened.
  template <int D1>
  __device__ __forceinline__ void take(const OrdHeap<ALGO, D1>& o) {
    widen(ta, o.ta);
    if constexpr (kKeys) widen(tb, o.tb);
    F = o.F; L = o.L; rover = o.rover;
    hd = o.hd; bm = o.bm; slb = o.slb; frl = o.frl; frh = o.frh;
  }
  template <typename T2, typename T1>
  __device__ __forceinline__ static void widen(T2& t, const T1& o) {
    t.init(o.lb, o.gb, o.nl_req);
#pragma unroll
    for (int k = 0; k < T1::ND; ++k) {
      t.dsl[k] = o.dsl[k]; t.dct[k] = o.dct[k]; t.dk0[k] = o.dk0[k]; t.dk1[k] = o.dk1[k];
      t.dmx[k] = o.dmx[k]; t.used[k] = o.used[k];
    }
    t.nc = o.nc;
  }

  // CHK = false: block_safe holds for the current block, so no request of
  // it finds a table at the directory's limit or reaches a capacity.
  template <bool CHK = true>
  __device__ __forceinline__ int64_t alloc(uint32_t sg, uint32_t kreq) {
    if (CHK && full_dir()) return kOverflow;
    if constexpr (ALGO == kFirstFit) {
      const uint32_t ci = ta.first_fit_chunk(sg, 0u);
      if (ci == kNone) return kFail;
      const Row r = ta.load(ta.slot(ci));
      const uint32_t p = ctz64(ballot(r.s >= sg));
      const uint32_t e = rdlane(r.a, p), s = rdlane(r.s, p);
      if (CHK && L >= capL) return kENoMeta;
      return commit_fit(ci, p, r, e, s, sg);
    } else if constexpr (ALGO == kNextFit) {
      // the search starts at the first block ending past the rover (R9-R11)
      // and runs on cyclically: the rest of that chunk, the later chunks,
      // then from the first chunk
      uint32_t ci0, p0;
      Row r0;
      ta.locate(0u, rover, ci0, r0, p0);
      uint32_t ci = kNone, p = 0;
      Row r;
      bool found = false;
      if (ci0 != kNone) {
        const uint64_t fit = ballot(r0.s >= sg) & lanes_below(ta.count(ci0)) & ~lanes_below(p0 + 1u);
        if (fit != 0ull) { ci = ci0; p = ctz64(fit); r = r0; found = true; }
      }
      if (!found) {
        const uint32_t c1 = ta.first_fit_chunk(sg, ci0 == kNone ? 0u : ci0 + 1u);
        const uint32_t c2 = c1 != kNone ? c1 : ta.first_fit_chunk(sg, 0u);
        if (c2 == kNone) return kFail;
        ci = c2;
        r = c2 == ci0 ? r0 : ta.load(ta.slot(c2));
        p = ctz64(ballot(r.s >= sg) & lanes_below(ta.count(c2)));
      }
      const uint32_t e = rdlane(r.a, p), s = rdlane(r.s, p);
      if (CHK && L >= capL) return kENoMeta;
      return commit_fit(ci, p, r, e, s, sg);
    } else if constexpr (ALGO == kBestFit) {
      // smallest key (size, end) at or above (sg, 0)
      uint32_t ci, p;
      typename TB::Row r;
      tb.insert_pos(sg, 0u, ci, r, p);
      if (p >= tb.count(ci)) {
        if (ci + 1u >= tb.nc) return kFail;
        ci = ci + 1u;
        r = tb.load(tb.slot(ci));
        p = 0u;
      }
      const uint32_t s = rdlane(r.s, p), e = rdlane(r.a, p);
      if (CHK && L >= capL) return kENoMeta;
      // the block's entry in the address table is looked up first: the key
      // table's updates do not touch it, and its load then overlaps them
      uint32_t cj, q;
      Row ra;
      ta.locate(0u, e, cj, ra, q);
      tb.erase_at(ci, p, r);
      if (s > sg) tb.insert_key(e, s - sg);
      return commit_fit(cj, q, ra, e, s, sg);
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
      const uint32_t i = head(c);
      const Rec b = rec(i);
      if (CHK && L >= capL) return kENoMeta;
      // pop the head (Alg. 4), keeping the lists' invariants (R20)
      set_head(c, b.nx);
      if (b.nx == kNone) bit_clear(c); else rec_link(b.nx, 3u, kNone);
      if (b.s > sg) {
        // the remainder, same record and same end, is pushed at the head of
        // its class (Alg. 4)
        push(i, b.a + sg, b.s - sg);
      } else {
        uint32_t ci, p;
        Row r;
        ta.locate(0u, b.a + b.s, ci, r, p);
        ta.erase_at(ci, p, r);
        rec_give(i);
        --F;
      }
      lset(L, mk_ent(b.a, sg));
      ++L;
      return (int64_t)((uint64_t)b.a << shift);
    }
  }

  // Release [x, x + sz) into the free blocks, merging with free neighbours
  // (Alg. 2 / Alg. 5).  Returns false, changing nothing, when a new free
  // entry would exceed the capacity.
  template <bool CHK = true>
  __device__ __forceinline__ bool release(uint32_t x, uint32_t sz) {
    const uint32_t lane = lane_id();
    const uint32_t xe = x + sz;
    // the block ending at x (an exact key) and the block after x (the next
    // entry, starting at xe if it borders)
    uint32_t ci, p;
    Row r;
    ta.locate(0u, x, ci, r, p);
    const bool hasL = ci != kNone && rdlane(r.a, p) == x;
    const uint32_t vl = ci != kNone ? rdlane(r.s, p) : 0u;  // size or record
    // the entry after position p of chunk ci (ci = kNone: the first entry)
    uint32_t rci = kNone, rp = 0;
    Row rr = r;
    if (ci != kNone && p + 1u < ta.count(ci)) {
      rci = ci; rp = p + 1u;
    } else {
      const uint32_t nci = ci == kNone ? 0u : ci + 1u;
      if (nci < ta.nc && ta.count(nci) != 0u) {
        rci = nci; rp = 0u;
        rr = ta.load(ta.slot(nci));
      }
    }
    const uint32_t er = rci != kNone ? rdlane(rr.a, rp) : 0u;
    const uint32_t vr = rci != kNone ? rdlane(rr.s, rp) : 0u;
    uint32_t sl = 0, sr = 0;
    Rec bl{0, 0, kNone, kNone}, br{0, 0, kNone, kNone};
    bool hasR;
    if constexpr (kSeg) {
      // both records are loaded before either is used
      const u32x4 ql = rec_raw(hasL ? vl : 0u), qr = rec_raw(rci != kNone ? vr : 0u);
      if (hasL) bl = rec_of(ql);
      if (rci != kNone) br = rec_of(qr);
      sl = bl.s;
      sr = br.s;
      hasR = rci != kNone && br.a == xe;
    } else {
      sl = vl;
      sr = vr;
      hasR = rci != kNone && er - vr == xe;
    }
    if (CHK && !hasL && !hasR && F >= capF) return false;
    const uint32_t ma = hasL ? x - sl : x;
    const uint32_t ms = (hasL ? sl : 0u) + sz + (hasR ? sr : 0u);
    const uint32_t me = hasR ? er : xe;  // end of the merged block
    if constexpr (kSeg) {
      // unlink the free neighbours, then push the merged block (R21)
      if (hasL) {
        unlink(sl, bl.nx, bl.pv);
        // unlinking the left block rewrote the links of its list
        // neighbours, which may include the right block
        br.pv = br.pv == vl ? bl.pv : br.pv;
        br.nx = br.nx == vl ? bl.nx : br.nx;
      }
      if (hasR) unlink(sr, br.nx, br.pv);
    }
    if constexpr (kKeys) {
      if (hasL) tb.erase_key(x, sl);
      if (hasR) tb.erase_key(er, sr);
      tb.insert_key(me, ms);
    }
    if (hasL && hasR) {
      // the right block's entry keeps its end and takes the merged block;
      // the left block's entry goes
      if constexpr (kSeg) {
        push(vr, ma, ms);
        rec_give(vl);
      } else {
        ta.store_field(ta.slot(rci), rp, 1u, ms);
        if (rci == ci) r = TA::with(r, rp, er, ms);  // the row erase_at shifts
        else if (kMax) dir_put(ta.dmx, rci, wave_max(TA::with(rr, rp, er, ms).s));
      }
      ta.erase_at(ci, p, r);
      --F;
    } else if (hasL) {
      // the left block's entry: end x -> xe (its place does not change)
      const uint32_t v = kSeg ? vl : ms;
      ta.store_entry(ta.slot(ci), p, xe, v);
      if (p == 0u) dir_put(ta.dk0, ci, xe);
      if (kMax) dir_put(ta.dmx, ci, wave_max(TA::with(r, p, xe, ms).s));
      if constexpr (kSeg) push(vl, ma, ms);
    } else if (hasR) {
      // the right block grows downwards: its end and its entry stay
      if constexpr (kSeg) {
        push(vr, ma, ms);
      } else {
        ta.store_field(ta.slot(rci), rp, 1u, ms);
        if (kMax) dir_put(ta.dmx, rci, wave_max(TA::with(rr, rp, er, ms).s));
      }
    } else {
      // a new entry right after position p (ci = kNone: first of chunk 0)
      uint32_t v = sz;
      if constexpr (kSeg) {
        v = rec_take();
        push(v, x, sz);
      }
      const uint32_t ic = ci == kNone ? 0u : ci, ip = ci == kNone ? 0u : p + 1u;
      const Row ir = ci == kNone ? (rci == 0u ? rr : ta.load(ta.slot(0u))) : r;
      ta.insert_at(ic, ip, ir, Row{xe, v});
      ++F;
    }
    (void)lane;
    return true;
  }

  // Free live entry idx except its first floor(cut * size / 2^31) granules
  // (partial deallocation, sequential fits; cut < 2^31).  Returns the byte
  // offset of the released part or kENoMeta.
  template <bool CHK = true>
  __device__ __forceinline__ int64_t free_index(uint32_t idx, uint32_t cut) {
    if (CHK && full_dir()) return kOverflow;
    const uint32_t last = L - 1u;
    // both entries are loaded before either is used, so their latencies
    // overlap
    const Ent v0 = lraw(idx), w0 = lraw(last);
    const Ent v = mk_ent(uniform(ent_a(v0)), uniform(ent_s(v0)));
    const Ent w = mk_ent(uniform(ent_a(w0)), uniform(ent_s(w0)));
    const uint32_t bx = ent_a(v), bsz = ent_s(v);
    const uint32_t t = (kSeg || cut == 0u) ? 0u : (uint32_t)(((uint64_t)cut * bsz) >> 31);
    const uint32_t x = bx + t, sz = bsz - t;
    if (!release<CHK>(x, sz)) return kENoMeta;
    if (t != 0u) {
      lset(idx, mk_ent(bx, t));
    } else {
      lset(idx, w);
      L = last;
    }
    return (int64_t)((uint64_t)x << shift);
  }

  template <bool CHK = true>
  __device__ __forceinline__ int64_t free_draw(uint32_t r, uint32_t cut) {
    if (CHK && L == 0u) return kFail;
    return free_index<CHK>((uint32_t)(((uint64_t)r * (uint64_t)L) >> 32), cut);
  }

  // Whether the next n requests can skip the directory and capacity checks:
  // each adds at most one live entry and one free block, so none of them
  // reaches a capacity, and with n live blocks to start from no free finds
  // the live table empty.  Every chunk of a table holds at least 32 entries
  // once there are two, so a table with fewer than 32 x 64 D free blocks has
  // fewer than 64 D chunks: with F + n below that, no request starts with a
  // table at the directory's limit.  (With the widest directory there is no
  // directory check.)
  __device__ __forceinline__ bool block_safe(uint32_t n) const {
    return L + n <= capL && F + n <= capF && L >= n &&
           (D >= kOrdDir || F + n < 32u * 64u * D);
  }
  __device__ __forceinline__ void set_room() {}  // nothing to refresh after a block

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
      uint32_t a = r.a - r.s, s = r.s;
      if constexpr (kSeg) {
        // this lane's record (lanes past the chunk read record 0, unused)
        wave_sync();
        const uint32_t i = lane < n && r.s < kOrdMaxFree ? r.s : 0u;
        u32x4 v;
        if (i < m.rec_n) v = m.rec_l[i]; else v = m.rec_g[i];
        a = v[0];
        s = v[1];
      }
      wave_sync();
      if (lane < n) {
        fo[2 * (k + lane)] = (int64_t)((uint64_t)a << sh);
        fo[2 * (k + lane) + 1] = (int64_t)((uint64_t)s << sh);
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
      // next links (bounded by the section's words even if a list were
      // corrupt)
      int64_t* ls = tail + 2;
      uint32_t pos = 0;
      for (uint32_t c = 0; c < (uint32_t)lists; ++c) {
        bool nonempty;
        if constexpr (ALGO == kTlsf) nonempty = (rdlane(slb, c >> 5) >> (c & 31u)) & 1u;
        else nonempty = (bm >> c) & 1ull;
        uint32_t n = 0;
        if (nonempty) {
          uint32_t i = head(c);
          while (i != kNone && pos + 1u + n < (uint32_t)lists + F) {
            const Rec b = rec(i);
            wave_sync();
            if (lane == 0) ls[pos + 1u + n] = (int64_t)((uint64_t)b.a << sh);
            i = b.nx;
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
