// One heap's replay by one wavefront: validate its parameters, initialise
// the tables (Alg. 6), run its requests in order and write results and the
// canonical state.  Shared by the persistent and the per-heap launches.
#pragma once
#include <stdint.h>

#include "hda_core.h"
#include "hda_lean.h"

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
  int32_t* ovf_list;     // heaps that outgrew the lean tiers (lean kernels append)
  uint32_t* ovf_count;   // their number
  int64_t n_heaps;       // heaps handled by this launch
  int64_t first;         // index into `order` of the first heap
  uint32_t cap_free, cap_live;   // total table capacities per heap
  uint32_t kf, kl;               // cold entries kept in LDS per wave
  uint32_t sf, sl;               // cold entries kept in device memory per wave
  uint32_t waves_per_group;
  uint32_t lds_wave_bytes;
  int use_queue;         // 1: pull heaps from the queue; 0: wave w takes heap w
};

// Validate heap parameters; on success fill the uniform heap registers.
__device__ __forceinline__ bool heap_params(const ReplayParams& p, int64_t heap, HeapRegs& h) {
  const int64_t A = p.arena[heap], g = p.align[heap];
  const int algo = p.algo[heap];
  if (algo < 0 || algo > 3 || g <= 0 || (g & (g - 1)) || A <= 0 || (A % g) ||
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

template <int ALGO, int RF, int RL>
__device__ void replay_heap(const ReplayParams& p, const Cold& c, const HeapRegs& regs,
                            int64_t heap) {
  const uint32_t lane = lane_id();
  const uint32_t hot_f = 64u * RF, hot_l = 64u * RL;
  const uint32_t capF = p.cap_free, capL = p.cap_live;
  WaveHeap<ALGO, RF, RL> w(c, regs, capF, capL);
  (void)hot_f; (void)hot_l;
  w.init();
  const int64_t b0 = p.req_off[heap], b1 = p.req_off[heap + 1];
  const uint64_t gm = (1ull << w.h.shift) - 1ull;
  // Requests are read 64 at a time (one per lane) and decoded by all lanes at
  // once: a free carries its draw, an allocation its size in granules (0 when
  // larger than the arena) and, for segregated fit, its byte class.  Loads are
  // clamped to the heap's last request instead of guarded by a lane-dependent
  // branch, since the values feed wave-wide reads.
  const int64_t last = b1 - 1;
  int64_t nxt = b1 > b0 ? p.req[min<int64_t>(b0 + lane, last)] : 0;
  for (int64_t base = b0; base < b1; base += 64) {
    const int64_t q = nxt;
    nxt = p.req[min<int64_t>(base + 64 + lane, last)];
    const bool is_free = q < 0;
    const bool big = q > w.h.arena;
    uint32_t sg = (uint32_t)(((uint64_t)q + gm) >> w.h.shift);
    sg = sg == 0u ? 1u : sg;
    const uint32_t w0 = is_free ? (uint32_t)~(uint64_t)q : (big ? 0u : sg);
    const uint32_t w1 = ceil_log2_u32(sg) + w.h.shift;
    const uint64_t mfree = ballot(is_free);
    const uint32_t n = (uint32_t)min<int64_t>(64, b1 - base);
    uint32_t olo = 0, ohi = 0;
    for (uint32_t j = 0; j < n; ++j) {
      const uint32_t v0 = rdlane(w0, j);
      int64_t r;
      if ((mfree >> j) & 1ull) {
        r = w.free_draw(v0);
      } else if (v0 == 0u) {
        r = kFail;
      } else {
        r = w.alloc(v0, ALGO == kSegFit ? rdlane(w1, j) : 0u);
      }
      if (r == kENoMeta && w.h.status == 0) w.h.status = (int32_t)kENoMeta;
      olo = put_lane(olo, j, (uint32_t)(uint64_t)r);
      ohi = put_lane(ohi, j, (uint32_t)((uint64_t)r >> 32));
    }
    if (base + lane < b1) p.res[base + lane] = (int64_t)(((uint64_t)ohi << 32) | olo);
  }
  int32_t st = w.h.status;
  if (p.state) {
    const int64_t so = p.state_off[heap], cap = p.state_off[heap + 1] - so;
    const int64_t need = w.dump(p.state + so, cap);
    if (lane == 0) p.state_len[heap] = need;
    if (need > cap && st == 0) st = (int32_t)kERange;
  }
  if (lane == 0) p.status[heap] = st;
}

// Lean path (hda_lean.h).  Returns false when the tables outgrew the fast
// tiers: then no state or status has been written, and the results written so
// far are to be overwritten by a replay on the general path.
template <int ALGO, int RF>
__device__ bool lean_replay_heap(const ReplayParams& p, const LeanLds& lds, const HeapRegs& regs,
                                 int64_t heap) {
  const uint32_t lane = lane_id();
  LeanHeap<ALGO, RF> w(lds, regs, p.cap_free, p.cap_live);
  w.init();
  int32_t st = 0;
  const int64_t b0 = p.req_off[heap], b1 = p.req_off[heap + 1];
  const uint64_t gm = (1ull << w.shift) - 1ull;
  const int64_t last = b1 - 1;
  int64_t nxt = b1 > b0 ? p.req[min<int64_t>(b0 + lane, last)] : 0;
  for (int64_t base = b0; base < b1; base += 64) {
    const int64_t q = nxt;
    nxt = p.req[min<int64_t>(base + 64 + lane, last)];
    const bool is_free = q < 0;
    const bool big = q > w.arena;
    uint32_t sg = (uint32_t)(((uint64_t)q + gm) >> w.shift);
    sg = sg == 0u ? 1u : sg;
    const uint32_t w0 = is_free ? (uint32_t)~(uint64_t)q : (big ? 0u : sg);
    const uint32_t w1 = ceil_log2_u32(sg) + w.shift;
    const uint64_t mfree = ballot(is_free);
    const uint32_t n = (uint32_t)min<int64_t>(64, b1 - base);
    uint32_t olo = 0, ohi = 0;
    for (uint32_t j = 0; j < n; ++j) {
      const uint32_t v0 = rdlane(w0, j);
      int64_t r;
      if ((mfree >> j) & 1ull) {
        r = w.free_draw(v0);
      } else if (v0 == 0u) {
        r = kFail;
      } else {
        r = w.alloc(v0, ALGO == kSegFit ? rdlane(w1, j) : 0u);
      }
      if (r == kOverflow) return false;
      if (r == kENoMeta && st == 0) st = (int32_t)kENoMeta;
      olo = put_lane(olo, j, (uint32_t)(uint64_t)r);
      ohi = put_lane(ohi, j, (uint32_t)((uint64_t)r >> 32));
    }
    if (base + lane < b1) p.res[base + lane] = (int64_t)(((uint64_t)ohi << 32) | olo);
  }
  if (p.state) {
    const int64_t so = p.state_off[heap], cap = p.state_off[heap + 1] - so;
    const int64_t need = w.dump(p.state + so, cap);
    if (lane == 0) p.state_len[heap] = need;
    if (need > cap && st == 0) st = (int32_t)kERange;
  }
  if (lane == 0) p.status[heap] = st;
  return true;
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

// Lean replay of one heap known to use algorithm ALGO; a heap that outgrows
// the fast tiers is appended to the overflow list.
template <int ALGO, int RF>
__device__ __forceinline__ void lean_one_heap(const ReplayParams& p, const LeanLds& lds,
                                              int64_t heap) {
  HeapRegs h;
  if (!heap_params(p, heap, h) || h.algo != ALGO) {
    reject_heap(p, heap);
    return;
  }
  if (!lean_replay_heap<ALGO, RF>(p, lds, h, heap)) {
    if (lane_id() == 0) p.ovf_list[atomicAdd(p.ovf_count, 1u)] = (int32_t)heap;
  }
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
    default: replay_heap<kSegFit, RF, RL>(p, c, h, heap); break;
  }
}

}  // namespace hda
