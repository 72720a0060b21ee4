// Batched replay of bitmask-allocator heaps (Sec. III-B; csrc/hda_bitmap.h):
// one wavefront per heap, each wave owning a workspace slot with the heap's
// granule flags and live table, waves taking heaps in turn.
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

// Workspace words of one wave's slot: the flags of max_granules, their node
// summaries (one per 64 words), then the live table.
__host__ __device__ uint64_t flag_words(uint64_t max_granules) { return (max_granules + 63u) / 64u; }
__host__ __device__ uint64_t node_words(uint64_t max_granules) { return (flag_words(max_granules) + 63u) / 64u; }
uint64_t slot_words(uint64_t max_granules, int64_t cap_live) {
  return flag_words(max_granules) + node_words(max_granules) + (uint64_t)cap_live;
}

int64_t n_waves(int64_t heaps) { return heaps < kMaxWaves ? heaps : kMaxWaves; }

__global__ __launch_bounds__(64 * kWavesPerGroup) void bitmap_kernel(ReplayParams p,
                                                                     uint64_t* ws,
                                                                     uint64_t max_granules,
                                                                     uint64_t words,
                                                                     int64_t waves) {
  const int64_t wave = uniform(blockIdx.x * kWavesPerGroup + threadIdx.x / 64u);
  if (wave >= waves) return;
  uint64_t* slot = ws + (uint64_t)wave * words;
  uint64_t* bits = slot;
  uint64_t* nodes = slot + flag_words(max_granules);
  Ent* live = reinterpret_cast<Ent*>(nodes + node_words(max_granules));
  for (int64_t i = wave; i < p.n_heaps; i += waves)
    bitmap_one_heap(p, bits, nodes, live, max_granules, p.order ? p.order[i] : i);
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
  return (size_t)(n_waves(d->n_heaps) * slot_words(max_granules, d->meta_live) * 8u) + 256u;
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
  hipLaunchKernelGGL(bitmap_kernel, dim3(groups), dim3(64 * kWavesPerGroup), 0,
                     static_cast<hipStream_t>(stream), p, reinterpret_cast<uint64_t*>(base),
                     max_granules, slot_words(max_granules, d->meta_live), waves);
  return hipGetLastError() == hipSuccess ? HDA_OK : HDA_E_DEVICE;
}

}  // extern "C"
