// Bitmask allocator with a next-fit search (Sec. III-B), one wavefront per
// heap.  The heap's metadata is one flag per granule (set = free), 64 to a
// word, in device memory, plus the live table the replay driver frees from.
// An allocation of s granules takes the first s free granules in a row found
// scanning from the rover (the end of the last allocation), else from granule
// 0, and moves the rover past them; a free sets the flags back, so merging is
// implicit.
//
// The flags are summarised per node of 64 words (4,096 granules): the free
// run at the node's bottom and the free run at its top, kept exact by every
// change of the flags, and a bound on the longest free run inside it.  A free
// recomputes the whole summary; an allocation only takes granules away, so
// it recomputes the two end runs and leaves the bound as it was (at least
// the true longest run).  A search that trusts a stale bound finds no run in
// that node's words, goes on past it with the exact end runs, and makes the
// node's summary exact again from the words it read.  A search reads the
// words of the rover's node (one word per lane), then the node summaries (one
// node per lane), which name the first node where a long enough run reaches
// its s-th granule, then that node's words: three dependent reads where a
// flag-only scan takes one per 4,096 granules.  Inside a step, the run
// reaching the bottom of a lane's word (or node) from below is found from the
// nearest lower lane that is not all free (a ballot, then a lane permute for
// that lane's top run); a run that reaches s inside a word is found with s-1
// shift-and steps.  The lowest start in the step is that of the lowest lane
// holding one (a ballot).
// Same rules as the other cores: values that feed a cross-lane operation are
// computed by all lanes with selects, never under a lane-dependent branch.
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

// Longest run of set bits in w.  y[k] marks the bits that start a run of at
// least 2^k; the length is then built from the top power down, keeping the
// starts that still reach it.
__device__ __forceinline__ uint32_t longest_run(uint64_t w) {
  uint64_t y[6];
  y[0] = w;
#pragma unroll
  for (int k = 1; k < 6; ++k) y[k] = y[k - 1] & (y[k - 1] >> (1u << (k - 1)));
  uint64_t z = ~0ull;  // starts of runs of at least len
  uint32_t len = 0;
#pragma unroll
  for (int k = 5; k >= 0; --k) {
    const uint64_t t = z & (y[k] >> len);  // len <= 62 here
    z = t ? t : z;
    len += t ? (1u << k) : 0u;
  }
  return w == ~0ull ? 64u : len;
}

constexpr uint32_t kNodeGranules = 4096;  // 64 words

// Node summary word: bottom run | top run << 16 | longest run << 32 (each
// 0..4096 granules; the longest run may be an upper bound).  0 = no free
// granule.
__device__ __forceinline__ uint32_t node_low(uint64_t r) { return (uint32_t)r & 0xffffu; }
__device__ __forceinline__ uint32_t node_top(uint64_t r) { return (uint32_t)(r >> 16) & 0xffffu; }
__device__ __forceinline__ uint32_t node_max(uint64_t r) { return (uint32_t)(r >> 32); }

// Summary of the node whose word `lane` is w (all lanes).  The longest run
// is the longest of the runs that reach a word boundary (they end at the
// bottom of the next word that is not all free, or at the node's top) and
// the runs inside single words; a word's inner runs are measured only when
// its free granules outnumber the longest boundary run.
__device__ __forceinline__ uint64_t node_summary(uint64_t w) {
  const uint32_t lane = lane_id();
  const bool full = w == ~0ull;
  const uint32_t low1 = full ? 64u : ctz64u(~w);
  const uint32_t top1 = full ? 64u : clz64u(~w);
  const uint64_t nf = ballot(!full);
  const uint64_t lt = nf & ((1ull << lane) - 1ull);
  const uint32_t ps = lt ? 63u - clz64u(lt) : 0u;
  const uint32_t tp = shfl(top1, ps);
  // free run ending just below this word, inside the node
  const uint32_t pre = lt ? tp + 64u * (lane - 1u - ps) : 64u * lane;
  const uint32_t topv = full ? pre + 64u : top1;  // free run ending at this word's top
  uint32_t m = full ? 0u : pre + low1;
  m = (lane == 63u && topv > m) ? topv : m;
  uint32_t mx = rdlane(wave_scan_max(m), 63u);
  if (ballot(!full && popc64(w) > mx)) {  // wave-uniform
    const uint32_t inner = rdlane(wave_scan_max(longest_run(w)), 63u);
    mx = inner > mx ? inner : mx;
  }
  const uint32_t fl = nf ? ctz64u(nf) : 0u;
  const uint32_t lw = rdlane(low1, fl);
  const uint32_t bottom = nf ? 64u * fl + lw : kNodeGranules;
  const uint32_t top = rdlane(topv, 63u);
  return (uint64_t)bottom | ((uint64_t)top << 16) | ((uint64_t)mx << 32);
}

// End runs of the node whose word `lane` is w (all lanes): bottom | top << 16,
// the low half of its summary word.
__device__ __forceinline__ uint32_t node_ends(uint64_t w) {
  const bool full = w == ~0ull;
  const uint32_t low1 = full ? 64u : ctz64u(~w);
  const uint32_t top1 = full ? 64u : clz64u(~w);
  const uint64_t nf = ballot(!full);
  const uint32_t fl = nf ? ctz64u(nf) : 0u;         // lowest word not all free
  const uint32_t hl = nf ? 63u - clz64u(nf) : 63u;  // highest
  const uint32_t bottom = nf ? 64u * fl + rdlane(low1, fl) : kNodeGranules;
  const uint32_t top = nf ? 64u * (63u - hl) + rdlane(top1, hl) : kNodeGranules;
  return bottom | (top << 16);
}

// The low half of a summary word is written through this type, which may
// alias the 64-bit word.
typedef uint32_t __attribute__((may_alias)) sum_half_t;

struct BitHeap {
  HDA_GLOBAL uint64_t* bits;   // nw words: bit i of word w = granule 64 w + i free
  HDA_GLOBAL uint64_t* nodes;  // nn node summaries, node n = words 64 n .. 64 n + 63
  HDA_GLOBAL Ent* live;        // capL entries
  // the first kn node summaries and the first kl live entries are kept in the
  // wave's LDS instead (the device-memory places of those stay unused)
  HDA_LDS uint64_t* lnodes;
  HDA_LDS Ent* llive;
  uint32_t kn, kl;
  int64_t arena;
  uint32_t shift, ag, nw, nn;
  uint32_t L, rover, capL;
  uint32_t cn;  // node whose words the last word step or mark left in cw, or kNone
  uint64_t cw;  // that node's word of this lane (no mask applied), always current:
                // only mark changes flags, and it updates cw

  __device__ __forceinline__ BitHeap(uint64_t* b, uint64_t* nd, Ent* lv, HDA_LDS uint64_t* lnd,
                                     uint32_t n_lds_nodes, HDA_LDS Ent* llv, uint32_t n_lds_live,
                                     const HeapRegs& h, uint32_t cap_live)
      : bits((HDA_GLOBAL uint64_t*)b), nodes((HDA_GLOBAL uint64_t*)nd),
        live((HDA_GLOBAL Ent*)lv), lnodes(lnd), llive(llv), kn(n_lds_nodes), kl(n_lds_live),
        arena(h.arena), shift(h.shift), ag(h.ag),
        nw((uint32_t)(((uint64_t)h.ag + 63u) >> 6)),  // ag may be 2^32 - 1
        nn((uint32_t)(((uint64_t)h.ag + 4095u) >> 12)), L(0), rover(0),
        capL(cap_live), cn(kNone), cw(0) {}

  // word wi, or 0 past the end (the load is clamped, not branched around)
  __device__ __forceinline__ uint64_t load(uint32_t wi) const {
    const uint64_t v = bits[wi < nw ? wi : nw - 1u];
    return wi < nw ? v : 0ull;
  }
  __device__ __forceinline__ uint64_t load_node(uint32_t ni) const {
    const uint32_t i = ni < nn ? ni : nn - 1u;
    wave_sync();
    const uint64_t v = i < kn ? lnodes[i] : nodes[i];
    return ni < nn ? v : 0ull;
  }
  __device__ __forceinline__ void put_node(uint32_t n, uint64_t v) const {
    wave_sync();
    if (n < kn) lnodes[n] = v;  // every lane, same value
    else if (lane_id() == 0u) nodes[n] = v;
  }
  // the end runs alone (the low half of node n's summary word)
  __device__ __forceinline__ void put_node_ends(uint32_t n, uint32_t v) const {
    wave_sync();
    if (n < kn) ((HDA_LDS sum_half_t*)lnodes)[2u * n] = v;  // every lane, same value
    else if (lane_id() == 0u) ((HDA_GLOBAL sum_half_t*)nodes)[2u * n] = v;
  }
  // live entry i (wave-uniform), as the same value in every lane
  __device__ __forceinline__ Ent live_get(uint32_t i) const {
    wave_sync();
    return i < kl ? llive[i] : live[i];
  }
  __device__ __forceinline__ void live_put(uint32_t i, Ent e) const {
    wave_sync();
    if (i < kl) llive[i] = e; else live[i] = e;  // every lane, same value
  }

  // Alg. 6: every granule free.
  __device__ void init() {
    for (uint32_t w0 = 0; w0 < nw; w0 += 64u) {
      const uint32_t wi = w0 + lane_id();
      const uint32_t rest = ag - 64u * (wi < nw ? wi : 0u);   // granules from this word on
      if (wi < nw) bits[wi] = rest >= 64u ? ~0ull : (1ull << rest) - 1ull;
    }
    for (uint32_t n0 = 0; n0 < nn; n0 += 64u) {
      const uint32_t ni = n0 + lane_id();
      const uint32_t rest = ag - kNodeGranules * (ni < nn ? ni : 0u);
      const uint32_t g = rest < kNodeGranules ? rest : kNodeGranules;  // one run [0, g)
      const uint32_t top = g == kNodeGranules ? g : 0u;
      const uint64_t v = (uint64_t)g | ((uint64_t)top << 16) | ((uint64_t)g << 32);
      wave_sync();
      if (ni < nn) {
        if (ni < kn) lnodes[ni] = v; else nodes[ni] = v;
      }
    }
    L = 0;
    rover = 0;
    cn = kNone;
  }

  // One step over node n's 64 words: the lowest p >= lo whose s-th granule
  // p + s - 1 lies in the node, with `carry` free granules in a row ending
  // just below the node (granules below lo count as used), or kNone; carry
  // becomes the free run ending at the node's top.
  // Run lengths and granule indexes are 32-bit: a run of free granules is
  // at most the arena's ag < 2^32 granules, and 64 wi < 2^32.
  __device__ __forceinline__ uint32_t word_step(uint32_t n, uint32_t lo, uint32_t s,
                                                uint32_t& carry) {
    const uint32_t lane = lane_id();
    const uint32_t wi = 64u * n + lane;
    const uint32_t lw = lo >> 6;
    const uint64_t below = wi < lw ? ~0ull : wi == lw ? (1ull << (lo & 63u)) - 1ull : 0ull;
    if (n != cn) {  // else cw holds the node's words as the last mark left them
      cw = load(wi);
      cn = n;
    }
    const uint64_t w = cw & ~below;
    const bool full = w == ~0ull;
    const uint32_t low1 = full ? 64u : ctz64u(~w);   // free run at the bottom
    const uint32_t top1 = full ? 64u : clz64u(~w);   // free run at the top
    const uint64_t lt = ballot(!full) & ((1ull << lane) - 1ull);
    const uint32_t ps = lt ? 63u - clz64u(lt) : 0u;
    const uint32_t tp = shfl(top1, ps);
    const uint32_t pre = lt ? tp + 64u * (lane - 1u - ps) : carry + 64u * lane;
    const uint32_t base = 64u * wi;
    // a run that reaches s in this word, having started below it
    uint32_t cand = (pre < s && pre + low1 >= s) ? base - pre : kNone;
    // a run of s inside this word
    if (s <= 64u) {
      uint64_t y = w;
      for (uint32_t k = 1; k < s;) {
        const uint32_t d = k < s - k ? k : s - k;
        y &= y >> d;
        k += d;
      }
      const uint32_t in = y ? base + ctz64u(y) : kNone;
      cand = in < cand ? in : cand;
    }
    const uint32_t topv = full ? pre + 64u : top1;
    carry = rdlane(topv, 63u);
    // Candidates rise with the lane: each starts s free granules that end in
    // its lane's word, and of two such runs the one ending in a lower word
    // cannot start later.  So the lowest lane with a candidate holds the
    // step's lowest start.
    const uint64_t hc = ballot(cand != kNone);
    return hc ? rdlane(cand, ctz64u(hc)) : kNone;
  }

  // The lowest p >= lo with granules [p, p + s) all free, or kNone.  Node
  // steps stop once they begin at or past below_end + s (only starts below
  // below_end are wanted then).  The summaries are read only once the word
  // step over the rover's node has found nothing, as most searches end there.
  __device__ uint32_t find(uint32_t lo, uint32_t s, uint64_t below_end = 1ull << 40) {
    const uint32_t lane = lane_id();
    uint32_t n1 = (lo >> 12) + 1u;
    uint32_t carry = 0;
    uint32_t K = word_step(lo >> 12, lo, s, carry);
    if (K != kNone) return K;
    uint64_t r = load_node(n1 + lane);
    while (n1 < nn && (uint64_t)kNodeGranules * n1 < below_end + s) {
      const uint32_t ni = n1 + lane;
      const uint32_t low1 = node_low(r), top1 = node_top(r);
      const bool full = low1 == kNodeGranules;
      const uint64_t lt = ballot(!full) & ((1ull << lane) - 1ull);
      const uint32_t ps = lt ? 63u - clz64u(lt) : 0u;
      const uint32_t tp = shfl(top1, ps);
      const uint32_t pre = lt ? tp + kNodeGranules * (lane - 1u - ps)
                              : carry + kNodeGranules * lane;
      // the first node where a run reaches its s-th granule
      const bool hit = (pre < s && pre + low1 >= s) || node_max(r) >= s;
      const uint64_t hb = ballot(hit && ni < nn);
      const uint32_t d = hb ? n1 + ctz64u(hb) : kNone;  // the lowest such node
      if (d != kNone) {
        uint32_t c2 = rdlane(pre, d - n1);
        K = word_step(d, 0u, s, c2);
        if (K != kNone) return K;
        // only a stale bound on d's longest run promises what d's words do
        // not hold: the summary is made exact from them (left in cw)
        put_node(d, node_summary(cw));
        carry = c2;
        n1 = d + 1u;
        r = load_node(n1 + lane);
        continue;
      }
      const uint32_t topv = full ? pre + kNodeGranules : top1;
      carry = rdlane(topv, 63u);
      n1 += 64u;
      r = load_node(n1 + lane);
    }
    return kNone;
  }

  // Granules [p, p + s) become free (set) or used (cleared), node by node:
  // each lane one word of the node (words a search or mark left in cw are reused),
  // then the node's summary (a free: all of it; an allocation: its end runs).
  __device__ void mark(uint32_t p, uint32_t s, bool set) {
    const uint32_t first = p >> 6, last = (p + s - 1u) >> 6;
    for (uint32_t n = p >> 12; n <= (last >> 6); ++n) {
      const uint32_t wi = 64u * n + lane_id();
      const bool in = wi >= first && wi <= last;
      // 32-bit: 64 wi and p + s stay below 2^32; for a word in the range
      // lo is 0..63 and e at least 1, and other words are masked off below
      const uint32_t b0 = 64u * wi;
      const uint32_t lo = p > b0 ? p - b0 : 0u;
      const uint32_t e = p + s - b0;
      const uint32_t hi = e < 64u ? e : 64u;
      const uint64_t m = in ? (hi == 64u ? ~0ull : (1ull << hi) - 1ull) & ~((1ull << (lo & 63u)) - 1ull)
                            : 0ull;
      uint64_t v;
      if (n == cn)
        v = cw;
      else
        v = load(wi);
      const uint64_t nv = set ? (v | m) : (v & ~m);
      if (in) bits[wi] = nv;
      cn = n;
      cw = nv;
      if (set)
        put_node(n, node_summary(nv));
      else
        put_node_ends(n, node_ends(nv));  // the longest run can only have shrunk
    }
  }

  // Allocate sg granules (sg >= 1).  Returns the byte offset, -1 or kENoMeta.
  // (CHK: no request of this core ends its run, so there is nothing to check)
  template <bool CHK = true>
  __device__ int64_t alloc(uint32_t sg, uint32_t) {
    if (sg > ag) return kFail;
    uint32_t p = find(rover, sg);
    // wrapping: starts at or past the rover were all tried
    if (p == kNone) p = find(0u, sg, rover);
    if (p == kNone) return kFail;
    if (L >= capL) return kENoMeta;
    mark(p, sg, false);
    live_put(L, mk_ent(p, sg));
    ++L;
    rover = p + sg;
    return (int64_t)((uint64_t)p << shift);
  }

  // Replay free: the victim is live[(r * L) >> 32]; it keeps its first
  // floor(cut * size / 2^31) granules (partial deallocation); nothing live
  // -> -1.  Returns the byte offset of the freed part.
  template <bool CHK = true>
  __device__ int64_t free_draw(uint32_t r, uint32_t cut) {
    if (L == 0u) return kFail;
    const uint32_t idx = (uint32_t)(((uint64_t)r * (uint64_t)L) >> 32);
    // both entries are read before either is used
    const Ent e = live_get(idx);
    const Ent last = live_get(L - 1u);
    const uint32_t x = uniform(ent_a(e)), sz = uniform(ent_s(e));
    const uint32_t t = cut == 0u ? 0u : (uint32_t)(((uint64_t)cut * sz) >> 31);
    mark(x + t, sz - t, true);
    if (t != 0u) {
      live_put(idx, mk_ent(x, t));
    } else {
      live_put(idx, mk_ent(uniform(ent_a(last)), uniform(ent_s(last))));
      --L;
    }
    return (int64_t)((uint64_t)(x + t) << shift);
  }

  // Every block may run without the run-ending checks of the other cores.
  __device__ __forceinline__ bool block_safe(uint32_t) const { return true; }
  __device__ __forceinline__ void set_room() {}

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
      const uint32_t j = i < L ? i : 0u;
      wave_sync();
      const Ent e = j < kl ? llive[j] : live[j];
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
