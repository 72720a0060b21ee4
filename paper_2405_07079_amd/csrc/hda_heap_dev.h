// Device-memory layout of a heap whose state persists between launches:
// a header holding the wave-uniform registers and the per-class counts,
// followed by the free table, its push stamps and the live table.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hda_core.h"

namespace hda {

struct HeapHdr {
  uint32_t F, L, ag, shift, rover, clock;
  int32_t algo, status;
  int64_t arena;
  uint32_t cf, cl;          // table capacities (multiples of 64)
  uint32_t pad[4];
  uint32_t cnt[64];         // free blocks per byte class
};
static_assert(sizeof(HeapHdr) % 16 == 0, "header keeps the tables 16 B aligned");

__host__ __device__ inline size_t heap_bytes(uint32_t cf, uint32_t cl) {
  return sizeof(HeapHdr) + (size_t)cf * 8 + (size_t)cf * 4 + (size_t)cl * 8;
}

__device__ inline Cold heap_cold(HeapHdr* hd) {
  uint8_t* base = reinterpret_cast<uint8_t*>(hd) + sizeof(HeapHdr);
  Cold c;
  c.lf = nullptr; c.lst = nullptr; c.ll = nullptr;  // no LDS part
  c.kf = 0; c.kl = 0;
  c.cf = hd->cf; c.cl = hd->cl;
  c.gf = (HDA_GLOBAL Ent*)(base);
  c.gst = (HDA_GLOBAL uint32_t*)(base + (size_t)c.cf * 8);
  c.gl = (HDA_GLOBAL Ent*)(base + (size_t)c.cf * 12);
  return c;
}

__device__ inline HeapRegs load_regs(const HeapHdr* hd) {
  HeapRegs h;
  h.F = hd->F; h.L = hd->L; h.ag = hd->ag; h.shift = hd->shift;
  h.rover = hd->rover; h.clock = hd->clock; h.algo = hd->algo; h.status = hd->status;
  h.arena = hd->arena;
  h.cnt = hd->cnt[lane_id()];
  return h;
}

__device__ inline void store_regs(HeapHdr* hd, const HeapRegs& h) {
  hd->cnt[lane_id()] = h.cnt;
  if (lane_id() == 0) {
    hd->F = h.F; hd->L = h.L; hd->rover = h.rover; hd->clock = h.clock;
    hd->status = h.status;
  }
}

}  // namespace hda
