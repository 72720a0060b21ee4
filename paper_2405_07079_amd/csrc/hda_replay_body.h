// One heap's replay by one wavefront: validate its parameters, initialise
// the tables (Alg. 6), run its requests in order and write results and the
// canonical state.  Shared by the persistent and the per-heap launches.
#pragma once
#include <stdint.h>

#include "hda_bitmap.h"
#include "hda_core.h"
#include "hda_lean.h"
#include "hda_ordered.h"

namespace hda {

struct ReplayParams {
  const int64_t* arena;
  const int64_t* align;
  const int32_t* algo;
  const int64_t* req_off;
  const int64_t* req;
  int64_t* res;
  const int32_t* order;
  int64_t* state;
  const int64_t* state_off;
  int64_t* state_len;
  int32_t* status;
  const int32_t* list;   // heaps this launch replays (one algorithm), or null
  const uint32_t* count; // number of heaps in `list` (device), or null
  uint32_t* queue;       // heap counter (persistent mode)
  Ent* spill_free;       // per wave slot: cold free entries past LDS
  uint32_t* spill_stamp; // per wave slot: their stamps
  Ent* spill_live;       // per wave slot: cold live entries past LDS
  uint32_t* migrated;    // heaps moved from the lean to the general core, or null
  int64_t n_heaps;       // heaps handled by this launch
  int64_t first;         // index into `order` of the first heap
  uint32_t cap_free, cap_live;   // total table capacities per heap
  uint32_t kf, kl;               // cold entries kept in LDS per wave
  uint32_t sf, sl;               // cold entries kept in device memory per wave
  uint32_t waves_per_group;
  uint32_t lds_wave_bytes;
  int use_queue;         // 1: pull heaps from the queue; 0: wave w takes heap w
  int64_t list_lo;       // queue mode: this launch takes list positions
  int64_t list_hi;       //   [list_lo, min(list_hi, *count))
  // ordered core (hda_ordered.h): per-wave LDS pool bytes, the part of it
  // meant for chunk slots, and the device slot of each wave
  uint32_t ord_pool_bytes;
  uint32_t ord_slot_bytes;
  uint8_t* ord_dev;
  uint64_t ord_dev_stride;
};

// Validate heap parameters; on success fill the uniform heap registers.
__device__ __forceinline__ bool heap_params(const ReplayParams& p, int64_t heap, HeapRegs& h) {
  const int64_t A = p.arena[heap], g = p.align[heap];
  const int algo = p.algo[heap];
  if (algo < 0 || algo > kBitmap || g <= 0 || (g & (g - 1)) || A <= 0 || (A % g) ||
      (A / g) >= (int64_t(1) << 32))
    return false;
  h.algo = algo;
  h.arena = A;
  h.shift = (uint32_t)__builtin_ctzll((uint64_t)g);
  h.ag = (uint32_t)(A >> h.shift);
  h.status = 0;
  h.F = h.L = h.rover = h.clock = h.cnt = 0;
  return true;
}

// Whether Core's blocks may run without the checks that end a core's run
// (the lean core's tiers, the ordered core's directory).
template <typename Core>
struct UncheckedBlocks {
  static constexpr bool value = false;
};
template <int A, int R>
struct UncheckedBlocks<LeanHeap<A, R>> {
  static constexpr bool value = true;
};
template <int A, int D>
struct UncheckedBlocks<OrdHeap<A, D>> {
  static constexpr bool value = true;
};
template <>
struct UncheckedBlocks<BitHeap> {
  static constexpr bool value = true;
};

// Requests j < n of one block of 64 on core w: lane j of w0 holds request
// j's draw (free) or size in granules (allocation, 0 = larger than the
// arena), lane j of w1 its byte class (segregated fit) or its cut (free,
// other fits; read only when CUT), bit j of mfree marks the frees.  Results
// go to lane j of olo / ohi.  Returns the number of requests run: n, or the
// index of the request that found the lean core's tiers too small.  UNCHK:
// the core's block_safe holds for the block, so no request can find the
// tiers (or the ordered core's directory) too small and the checks are
// compiled out.
template <int ALGO, bool CUT, bool UNCHK, typename Core>
__device__ __forceinline__ uint32_t run_block(Core& w, uint32_t n, uint32_t w0, uint32_t w1,
                                              uint64_t mfree, uint32_t& olo, uint32_t& ohi,
                                              int32_t& st) {
  uint32_t done = n;
  for (uint32_t j = 0; j < n; ++j) {
    const uint32_t v0 = rdlane(w0, j);
    int64_t r;
    if ((mfree >> j) & 1ull) {
      if constexpr (UNCHK) r = w.template free_draw<false>(v0, CUT ? rdlane(w1, j) : 0u);
      else r = w.free_draw(v0, CUT ? rdlane(w1, j) : 0u);
    } else if (v0 == 0u) {
      r = kFail;
    } else {
      if constexpr (UNCHK) r = w.template alloc<false>(v0, seg_like(ALGO) ? rdlane(w1, j) : 0u);
      else r = w.alloc(v0, seg_like(ALGO) ? rdlane(w1, j) : 0u);
    }
    if (!UNCHK && r == kOverflow) { done = j; break; }
    olo = put_lane(olo, j, (uint32_t)(uint64_t)r);
    ohi = put_lane(ohi, j, (uint32_t)((uint64_t)r >> 32));
  }
  // the heap's status: its first capacity error, looked for once per block
  // rather than once per request
  const bool nometa = lane_id() < done && olo == (uint32_t)(uint64_t)kENoMeta &&
                      ohi == (uint32_t)((uint64_t)kENoMeta >> 32);
  if (st == 0 && ballot(nometa) != 0ull) st = (int32_t)kENoMeta;
  return done;
}

// Run requests [from, to) of `heap` on core w (either core type).  Requests
// are read 64 at a time (one per lane) and decoded by all lanes at once: a
// free carries its draw and, for the sequential fits, its cut (the fraction
// of the victim kept live, partial deallocation), an allocation its size in
// granules (0 when larger than the arena) and, for segregated fit, its byte
// class.  Loads are clamped
// to the heap's last request instead of guarded by a lane-dependent branch,
// since the values feed wave-wide reads.  Returns the position of the first
// request not run: `to`, or the request that found the lean core's tiers too
// small (it changed nothing, and the results before it are stored).
template <int ALGO, typename Core>
__device__ __forceinline__ int64_t run_requests(const ReplayParams& p, Core& w, int64_t from, int64_t to,
                                uint32_t shift, int64_t arena, int32_t& st) {
  const uint32_t lane = lane_id();
  const uint64_t gm = (1ull << shift) - 1ull;
  const int64_t last = to - 1;
  int64_t nxt = to > from ? p.req[min<int64_t>(from + lane, last)] : 0;
  for (int64_t base = from; base < to; base += 64) {
    const int64_t q = nxt;
    nxt = p.req[min<int64_t>(base + 64 + lane, last)];
    const bool is_free = q < 0;
    const bool big = q > arena;
    uint32_t sg = (uint32_t)(((uint64_t)q + gm) >> shift);
    sg = sg == 0u ? 1u : sg;
    const uint32_t w0 = is_free ? (uint32_t)~(uint64_t)q : (big ? 0u : sg);
    // segregated fit: the byte class; TLSF: the request class; the other
    // fits: a free's cut
    const uint32_t w1 = ALGO == kSegFit ? ceil_log2_u32(sg) + shift
                      : ALGO == kTlsf   ? tlsf_request_class(sg, shift)
                                        : (is_free ? (uint32_t)(~(uint64_t)q >> 32) : 0u);
    const uint64_t mfree = ballot(is_free);
    const uint32_t n = (uint32_t)min<int64_t>(64, to - base);
    uint32_t olo = 0, ohi = 0;
    // a block whose frees carry no cut runs a copy with the partial-free
    // logic folded away; on the lean and ordered cores, such a block that
    // cannot outgrow the tiers (the directory) also runs without the checks
    const bool cut = !seg_like(ALGO) && ballot(is_free && w1 != 0u) != 0ull;
    uint32_t done;
    if (cut) {
      // (a partial free adds at most one free entry and keeps its live
      // entry, so the block test holds for these blocks too)
      if constexpr (UncheckedBlocks<Core>::value) {
        if (w.block_safe(n)) {
          done = run_block<ALGO, !seg_like(ALGO), true>(w, n, w0, w1, mfree, olo, ohi, st);
          w.set_room();
        } else {
          done = run_block<ALGO, !seg_like(ALGO), false>(w, n, w0, w1, mfree, olo, ohi, st);
        }
      } else {
        done = run_block<ALGO, !seg_like(ALGO), false>(w, n, w0, w1, mfree, olo, ohi, st);
      }
    } else if constexpr (UncheckedBlocks<Core>::value) {
      if (w.block_safe(n)) {
        done = run_block<ALGO, false, true>(w, n, w0, w1, mfree, olo, ohi, st);
        w.set_room();
      } else {
        done = run_block<ALGO, false, false>(w, n, w0, w1, mfree, olo, ohi, st);
      }
    } else {
      done = run_block<ALGO, false, false>(w, n, w0, w1, mfree, olo, ohi, st);
    }
    if (lane < done) p.res[base + lane] = (int64_t)(((uint64_t)ohi << 32) | olo);
    if (done < n) return base + done;
  }
  return to;
}

// Canonical state and status of a finished heap.
template <typename Core>
__device__ __forceinline__ void finish_heap(const ReplayParams& p, Core& w, int64_t heap,
                                            int32_t st) {
  if (p.state) {
    const int64_t so = p.state_off[heap], cap = p.state_off[heap + 1] - so;
    const int64_t need = w.dump(p.state + so, cap);
    if (lane_id() == 0) p.state_len[heap] = need;
    if (need > cap && st == 0) st = (int32_t)kERange;
  }
  if (lane_id() == 0) p.status[heap] = st;
}

template <int ALGO, int RF, int RL>
__device__ __forceinline__ void replay_heap(const ReplayParams& p, const Cold& c, const HeapRegs& regs,
                            int64_t heap) {
  WaveHeap<ALGO, RF, RL> w(c, regs, p.cap_free, p.cap_live);
  w.init();
  int32_t st = 0;
  run_requests<ALGO>(p, w, p.req_off[heap], p.req_off[heap + 1], w.h.shift, w.h.arena, st);
  finish_heap(p, w, heap, st);
}

// Lean path (hda_lean.h).  A heap whose tables outgrow the lean tiers moves
// them into the general core's layout -- the same LDS bytes, then the wave's
// device-memory spill slot -- and continues there from the request that
// did not fit.
template <int ALGO, int RF>
__device__ void lean_replay_heap(const ReplayParams& p, const LeanLds& lds, const Cold& c,
                                 const HeapRegs& regs, int64_t heap) {
  LeanHeap<ALGO, RF> w(lds, regs, p.cap_free, p.cap_live);
  w.init();
  int32_t st = 0;
  const int64_t b1 = p.req_off[heap + 1];
  const int64_t pos = run_requests<ALGO>(p, w, p.req_off[heap], b1, w.shift, w.arena, st);
  if (pos == b1) {
    finish_heap(p, w, heap, st);
    return;
  }
  WaveHeap<ALGO, 0, 0> g(c, regs, p.cap_free, p.cap_live);
  w.migrate(c, g.h);
  if (lane_id() == 0 && p.migrated) atomicAdd(p.migrated, 1u);
  run_requests<ALGO>(p, g, pos, b1, g.h.shift, g.h.arena, st);
  finish_heap(p, g, heap, st);
}

// Heap with invalid parameters: every result and the status are E_INVAL.
__device__ __forceinline__ void reject_heap(const ReplayParams& p, int64_t heap) {
  const uint32_t lane = lane_id();
  const int64_t b0 = p.req_off[heap], b1 = p.req_off[heap + 1];
  for (int64_t base = b0; base < b1; base += 64)
    if (base + lane < b1) p.res[base + lane] = kEInval;
  if (lane == 0) {
    p.status[heap] = (int32_t)kEInval;
    if (p.state_len) p.state_len[heap] = 0;
  }
}

// Replay one heap known to use algorithm ALGO (its parameters are checked
// again; a heap that fails the check is rejected).
template <int ALGO, int RF, int RL>
__device__ __forceinline__ void replay_one_heap(const ReplayParams& p, const Cold& c, int64_t heap) {
  HeapRegs h;
  if (!heap_params(p, heap, h) || h.algo != ALGO) {
    reject_heap(p, heap);
    return;
  }
  replay_heap<ALGO, RF, RL>(p, c, h, heap);
}

// Lean replay of one heap known to use algorithm ALGO.
template <int ALGO, int RF>
__device__ __forceinline__ void lean_one_heap(const ReplayParams& p, const LeanLds& lds,
                                              const Cold& c, int64_t heap) {
  HeapRegs h;
  if (!heap_params(p, heap, h) || h.algo != ALGO) {
    reject_heap(p, heap);
    return;
  }
  lean_replay_heap<ALGO, RF>(p, lds, c, h, heap);
}

// Any algorithm (used where one program must serve every heap).
template <int RF, int RL>
__device__ void replay_any_heap(const ReplayParams& p, const Cold& c, int64_t heap) {
  HeapRegs h;
  if (!heap_params(p, heap, h)) {
    reject_heap(p, heap);
    return;
  }
  switch (h.algo) {
    case kFirstFit: replay_heap<kFirstFit, RF, RL>(p, c, h, heap); break;
    case kNextFit: replay_heap<kNextFit, RF, RL>(p, c, h, heap); break;
    case kBestFit: replay_heap<kBestFit, RF, RL>(p, c, h, heap); break;
    case kSegFit: replay_heap<kSegFit, RF, RL>(p, c, h, heap); break;
    case kTlsf: replay_heap<kTlsf, RF, RL>(p, c, h, heap); break;
    default: reject_heap(p, heap); break;  // the bitmask allocator has its own kernel
  }
}

// Ordered core (hda_ordered.h) for one heap: tables in the wave's LDS pool
// and, past it, in its device slot.
template <int ALGO>
__device__ __forceinline__ void ord_replay_heap(const ReplayParams& p, HDA_LDS uint8_t* pool,
                                HDA_GLOBAL uint8_t* dev, const HeapRegs& regs, int64_t heap) {
  const OrdMem m = ord_mem(ALGO, pool, p.ord_pool_bytes, p.ord_slot_bytes, dev, p.cap_live);
  // one directory register while the tables fit 64 chunks, then two
  OrdHeap<ALGO, 1> w(m, regs, p.cap_free, p.cap_live);
  w.init();
  int32_t st = 0;
  const int64_t b1 = p.req_off[heap + 1];
  const int64_t pos = run_requests<ALGO>(p, w, p.req_off[heap], b1, regs.shift, regs.arena, st);
  if (pos == b1) {
    finish_heap(p, w, heap, st);
    return;
  }
  OrdHeap<ALGO, kOrdDir> w2(m, regs, p.cap_free, p.cap_live);
  w2.take(w);
  run_requests<ALGO>(p, w2, pos, b1, regs.shift, regs.arena, st);
  finish_heap(p, w2, heap, st);
}

__device__ __forceinline__ void ord_any_heap(const ReplayParams& p, HDA_LDS uint8_t* pool,
                                             HDA_GLOBAL uint8_t* dev, int64_t heap) {
  HeapRegs h;
  if (!heap_params(p, heap, h)) {
    reject_heap(p, heap);
    return;
  }
  switch (h.algo) {
    case kFirstFit: ord_replay_heap<kFirstFit>(p, pool, dev, h, heap); break;
    case kNextFit: ord_replay_heap<kNextFit>(p, pool, dev, h, heap); break;
    case kBestFit: ord_replay_heap<kBestFit>(p, pool, dev, h, heap); break;
    case kSegFit: ord_replay_heap<kSegFit>(p, pool, dev, h, heap); break;
    case kTlsf: ord_replay_heap<kTlsf>(p, pool, dev, h, heap); break;
    default: reject_heap(p, heap); break;  // the bitmask allocator has its own kernel
  }
}

// Bitmask-allocator replay of one heap (hda_bitmap.h) in a workspace slot
// of max_granules flags, their node summaries and p.cap_live live entries
// (the first kn summaries and kl live entries in the wave's LDS instead); a
// heap of another algorithm or a larger arena is rejected.
__device__ __forceinline__ void bitmap_one_heap(const ReplayParams& p, uint64_t* bits,
                                                uint64_t* nodes, Ent* live,
                                                HDA_LDS uint64_t* lnodes, uint32_t kn,
                                                HDA_LDS Ent* llive, uint32_t kl,
                                                uint64_t max_granules, int64_t heap) {
  HeapRegs h;
  if (!heap_params(p, heap, h) || h.algo != kBitmap || (uint64_t)h.ag > max_granules) {
    reject_heap(p, heap);
    return;
  }
  BitHeap w(bits, nodes, live, lnodes, kn, llive, kl, h, p.cap_live);
  w.init();
  int32_t st = 0;
  run_requests<kBitmap>(p, w, p.req_off[heap], p.req_off[heap + 1], h.shift, h.arena, st);
  finish_heap(p, w, heap, st);
}

}  // namespace hda
