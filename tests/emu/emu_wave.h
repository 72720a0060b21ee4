// Lockstep emulation of a 64-lane wavefront on the CPU.  The 64 lanes are
// user-level fibers on one host thread; every cross-lane primitive and every
// table access is a sync point at which a lane hands over to the next one, so
// lanes run the core's instructions in the order the hardware would: between
// two sync points each lane runs its own straight-line code, and whatever one
// lane wrote before a sync point is seen by all lanes after it.  Cross-lane
// values travel through a per-wave exchange array.
#pragma once
#include <ucontext.h>

#include <cstdint>

#include "hip/hip_runtime.h"

#define HDA_LDS
#define HDA_GLOBAL

namespace hda {

struct EmuWave {
  ucontext_t lane_ctx[64];
  ucontext_t main_ctx;
  uint64_t xch[64];
  uint64_t syncs = 0;
};

extern EmuWave* emu_wave;
extern uint32_t emu_lane;

inline uint32_t lane_id() { return emu_lane; }

// Hand over to the next lane; lane 63 hands back to lane 0, which completes
// one round (every lane has reached this sync point).
inline void wave_sync() {
  const uint32_t me = emu_lane, next = (me + 1) & 63u;
  if (me == 63) emu_wave->syncs++;
  emu_lane = next;
  swapcontext(&emu_wave->lane_ctx[me], &emu_wave->lane_ctx[next]);
  emu_lane = me;
}

template <typename F>
inline auto exchange(uint64_t v, F&& f) {
  wave_sync();
  emu_wave->xch[emu_lane] = v;
  wave_sync();
  auto r = f(emu_wave->xch);
  wave_sync();
  return r;
}

inline uint64_t ballot(bool p) {
  return exchange(p ? 1u : 0u, [](const uint64_t* x) {
    uint64_t m = 0;
    for (int i = 0; i < 64; ++i) m |= (x[i] & 1u) << i;
    return m;
  });
}

inline uint32_t rdlane(uint32_t v, uint32_t l) {
  return exchange(v, [l](const uint64_t* x) { return (uint32_t)x[l & 63u]; });
}

// writelane: only the lane's own register changes, no exchange needed
inline uint32_t put_lane(uint32_t v, uint32_t l, uint32_t x) {
  return emu_lane == (l & 63u) ? x : v;
}

// optimisation barrier on the GPU; nothing to do here
inline uint32_t opaque(uint32_t v) { return v; }

// a wait for a device-memory load on the GPU; nothing to do here
inline void settle(uint32_t) {}

// the first active lane; in the core this is only used with all lanes active
inline uint32_t uniform(uint32_t v) { return rdlane(v, 0); }

template <int K>
inline uint32_t row_shr(uint32_t old, uint32_t src) {
  const uint32_t me = emu_lane;
  return exchange(src, [me, old](const uint64_t* x) {
    return (me & 15u) >= (uint32_t)K ? (uint32_t)x[me - K] : old;
  });
}

// Rows 1 and 3 receive lane 15 of the row below (lanes 15 and 47); rows 0
// and 2 keep `old`.
inline uint32_t row_bcast15(uint32_t old, uint32_t src) {
  const uint32_t me = emu_lane;
  return exchange(src, [me, old](const uint64_t* x) {
    const uint32_t row = me >> 4;
    return (row & 1u) ? (uint32_t)x[16u * row - 1u] : old;
  });
}

// Rows 2 and 3 receive lane 31; rows 0 and 1 keep `old`.
inline uint32_t row_bcast31(uint32_t old, uint32_t src) {
  const uint32_t me = emu_lane;
  return exchange(src, [me, old](const uint64_t* x) {
    return (me >> 4) >= 2u ? (uint32_t)x[31] : old;
  });
}

// Whole-wave shifts by one lane; the lane with no source receives `old`.
inline uint32_t wave_shr1(uint32_t old, uint32_t src) {
  const uint32_t me = emu_lane;
  return exchange(src, [me, old](const uint64_t* x) { return me >= 1u ? (uint32_t)x[me - 1u] : old; });
}
inline uint32_t wave_shl1(uint32_t old, uint32_t src) {
  const uint32_t me = emu_lane;
  return exchange(src, [me, old](const uint64_t* x) { return me <= 62u ? (uint32_t)x[me + 1u] : old; });
}

inline uint32_t shfl(uint32_t v, uint32_t src_lane) {
  return exchange(v, [src_lane](const uint64_t* x) { return (uint32_t)x[src_lane & 63u]; });
}

}  // namespace hda
