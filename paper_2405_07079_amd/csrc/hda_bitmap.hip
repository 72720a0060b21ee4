// Batched replay of bitmask-allocator heaps (Sec. III-B; csrc/hda_bitmap.h):
// one wavefront per heap, each wave owning a workspace slot with the heap's
// granule flags, node summaries and live table (the first summaries and live
// entries in the wave's share of LDS), waves pulling heaps from a queue in
// the caller's order.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "hda.h"
#include "hda_wave.h"
#include "hda_core.h"
#include "hda_replay_body.h"

using namespace hda;

namespace {

constexpr uint32_t kWavesPerGroup = 4;
constexpr int64_t kMaxWaves = 4096;
// LDS per wave: the summaries of the first kLdsNodes nodes (a 16 MiB heap of
// 64 B granules has 64) and the first kLdsLive live entries
constexpr uint32_t kLdsNodes = 64, kLdsLive = 1024;
constexpr uint32_t kLdsWaveBytes = (kLdsNodes + kLdsLive) * 8u;
// the workspace starts with the heap queue's counter (256 bytes)
constexpr uint64_t kHeaderBytes = 256;

// Workspace words of one wave's slot: the flags of max_granules, their node
// summaries (one per 64 words), then the live table.
__host__ __device__ uint64_t flag_words(uint64_t max_granules) { return (max_granules + 63u) / 64u; }
__host__ __device__ uint64_t node_words(uint64_t max_granules) { return (flag_words(max_granules) + 63u) / 64u; }
uint64_t slot_words(uint64_t max_granules, int64_t cap_live) {
  return flag_words(max_granules) + node_words(max_granules) + (uint64_t)cap_live;
}

int64_t n_waves(int64_t heaps) { return heaps < kMaxWaves ? heaps : kMaxWaves; }

// The queue counter starts at 0 (a kernel rather than a memset, so the pair
// of launches can be captured in a graph).
__global__ void bitmap_reset(uint32_t* queue) {
  if (threadIdx.x == 0) *queue = 0u;
}

__global__ __launch_bounds__(64 * kWavesPerGroup) void bitmap_kernel(ReplayParams p,
                                                                     uint64_t* ws,
                                                                     uint64_t max_granules,
                                                                     uint64_t words,
                                                                     int64_t waves) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const uint32_t wl = uniform(threadIdx.x / 64u);
  const int64_t wave = uniform(blockIdx.x * kWavesPerGroup + wl);
  if (wave >= waves) return;
  uint32_t* queue = reinterpret_cast<uint32_t*>(ws);
  uint64_t* slot = ws + kHeaderBytes / 8u + (uint64_t)wave * words;
  uint64_t* bits = slot;
  uint64_t* nodes = slot + flag_words(max_granules);
  Ent* live = reinterpret_cast<Ent*>(nodes + node_words(max_granules));
  HDA_LDS uint8_t* mine = (HDA_LDS uint8_t*)smem + (size_t)wl * kLdsWaveBytes;
  HDA_LDS uint64_t* lnodes = (HDA_LDS uint64_t*)mine;
  HDA_LDS Ent* llive = (HDA_LDS Ent*)(mine + kLdsNodes * 8u);
  // a wave takes at most every heap, so the loop ends even if the queue were
  // never to run dry; every lane runs the atomic (lane 0 adds 1) so the value
  // read back does not come from a lane-dependent branch
  for (int64_t taken = 0; taken < p.n_heaps; ++taken) {
    uint32_t i = atomicAdd(queue, lane_id() == 0 ? 1u : 0u);
    i = rdlane(i, 0);
    if ((int64_t)i >= p.n_heaps) break;
    bitmap_one_heap(p, bits, nodes, live, lnodes, kLdsNodes, llive, kLdsLive, max_granules,
                    p.order ? p.order[i] : (int64_t)i);
  }
}

bool desc_ok(const hda_batch_desc* d, uint64_t max_granules) {
  if (!d || d->n_heaps < 0 || max_granules == 0 || max_granules >= (uint64_t(1) << 32) ||
      d->meta_live <= 0 || d->meta_live > (int64_t(1) << 31))
    return false;
  if (d->n_heaps == 0) return true;
  if (!d->arena || !d->align || !d->algo || !d->req_off || !d->req || !d->res || !d->status)
    return false;
  if (d->state && (!d->state_off || !d->state_len)) return false;
  return true;
}

}  // namespace

extern "C" {

size_t hda_bitmap_workspace(const hda_batch_desc* d, uint64_t max_granules) {
  if (!desc_ok(d, max_granules)) return 0;
  return (size_t)(n_waves(d->n_heaps) * slot_words(max_granules, d->meta_live) * 8u) +
         kHeaderBytes + 256u;
}

int hda_bitmap_replay(const hda_batch_desc* d, uint64_t max_granules, void* stream) {
  if (!desc_ok(d, max_granules)) return HDA_E_INVAL;
  if (d->n_heaps == 0) return HDA_OK;
  const size_t need = hda_bitmap_workspace(d, max_granules);
  if (!d->workspace || d->workspace_bytes < need) return HDA_E_RANGE;
  ReplayParams p;
  std::memset(&p, 0, sizeof(p));
  p.arena = d->arena; p.align = d->align; p.algo = d->algo;
  p.req_off = d->req_off; p.req = d->req; p.res = d->res; p.order = d->order;
  p.state = d->state; p.state_off = d->state_off; p.state_len = d->state_len;
  p.status = d->status;
  p.n_heaps = d->n_heaps;
  p.cap_live = (uint32_t)d->meta_live;
  const int64_t waves = n_waves(d->n_heaps);
  const uint32_t groups = (uint32_t)((waves + kWavesPerGroup - 1) / kWavesPerGroup);
  uintptr_t base = reinterpret_cast<uintptr_t>(d->workspace);
  base = (base + 255u) & ~uintptr_t(255);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(bitmap_reset, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(base));
  if (hipGetLastError() != hipSuccess) return HDA_E_DEVICE;
  hipLaunchKernelGGL(bitmap_kernel, dim3(groups), dim3(64 * kWavesPerGroup),
                     kLdsWaveBytes * kWavesPerGroup, s, p, reinterpret_cast<uint64_t*>(base),
                     max_granules, slot_words(max_granules, d->meta_live), waves);
  return hipGetLastError() == hipSuccess ? HDA_OK : HDA_E_DEVICE;
}

}  // extern "C"
