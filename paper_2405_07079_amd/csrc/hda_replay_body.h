// One heap's replay by one wavefront: validate its parameters, initialise
// the tables (Alg. 6), run its requests in order and write results and the
// canonical state.  Shared by the persistent and the per-heap launches.
#pragma once
#include <stdint.h>

#include "hda_core.h"

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
  uint32_t* queue;       // heap counter (persistent mode)
  Ent* spill_free;       // per wave slot: cf-kf entries
  uint32_t* spill_stamp; // per wave slot: cf-kf stamps
  Ent* spill_live;       // per wave slot: cl-kl entries
  int64_t n_heaps;       // heaps handled by this launch
  int64_t first;         // index into `order` of the first heap
  uint32_t kf, kl, cf, cl;
  uint32_t waves_per_group;
  uint32_t lds_wave_bytes;
  int use_queue;         // 1: pull heaps from the queue; 0: wave w takes heap w
};

// Validate heap parameters; on success fill the uniform heap registers.
__device__ bool heap_params(const ReplayParams& p, int64_t heap, HeapRegs& h) {
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
  return true;
}

__device__ void replay_one_heap(const ReplayParams& p, const Tables& t, int64_t heap) {
  const uint32_t lane = lane_id();
  const int64_t b0 = p.req_off[heap], b1 = p.req_off[heap + 1];
  HeapRegs h;
  if (!heap_params(p, heap, h)) {
    for (int64_t base = b0; base < b1; base += 64)
      if (base + lane < b1) p.res[base + lane] = kEInval;
    if (lane == 0) {
      p.status[heap] = (int32_t)kEInval;
      if (p.state_len) p.state_len[heap] = 0;
    }
    return;
  }
  heap_init(t, h);
  // Requests are read 64 at a time (one per lane) and handed out in order
  // with readlane; results collect in the lane of their slot and are written
  // back 64 at a time.  The next chunk is prefetched while this one runs.
  // Loads are clamped to the heap's last request instead of guarded by a
  // lane-dependent branch, since the values feed wave-wide reads.
  const int64_t last = b1 - 1;
  int64_t nxt = b1 > b0 ? p.req[min<int64_t>(b0 + lane, last)] : 0;
  for (int64_t base = b0; base < b1; base += 64) {
    const int64_t cur = nxt;
    nxt = p.req[min<int64_t>(base + 64 + lane, last)];
    const uint32_t qlo = (uint32_t)cur, qhi = (uint32_t)((uint64_t)cur >> 32);
    const uint32_t n = (uint32_t)min<int64_t>(64, b1 - base);
    int64_t out = 0;
    for (uint32_t j = 0; j < n; ++j) {
      const int64_t q = (int64_t)(((uint64_t)rdlane(qhi, j) << 32) | rdlane(qlo, j));
      const int64_t r = op_request(t, h, q);
      if (r == kENoMeta && h.status == 0) h.status = (int32_t)kENoMeta;
      out = (lane == j) ? r : out;
    }
    if (base + lane < b1) p.res[base + lane] = out;
  }
  int32_t st = h.status;
  if (p.state) {
    const int64_t so = p.state_off[heap], cap = p.state_off[heap + 1] - so;
    const int64_t need = dump_state(t, h, p.state + so, cap);
    if (lane == 0) p.state_len[heap] = need;
    if (need > cap && st == 0) st = (int32_t)kERange;
  }
  if (lane == 0) p.status[heap] = st;
}

}  // namespace hda
