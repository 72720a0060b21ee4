// Batched replay of many independent heaps on gfx950: one persistent launch,
// one wavefront per heap, heaps pulled from a device queue in the caller's
// order (longest trace first is the useful order for uneven batches).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "hda.h"
#include "hda_wave.h"
#include "hda_core.h"
#include "hda_replay_body.h"

using namespace hda;

namespace {

__global__ void reset_queue(uint32_t* q) { *q = 0u; }

__global__ void __launch_bounds__(1024) replay_kernel(ReplayParams p) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const uint32_t wave = threadIdx.x >> 6;
  HDA_LDS uint8_t* mine = (HDA_LDS uint8_t*)smem + (size_t)wave * p.lds_wave_bytes;
  const uint64_t slot = (uint64_t)blockIdx.x * p.waves_per_group + wave;
  Tables t;
  t.lf = (HDA_LDS Ent*)(mine);
  t.lst = (HDA_LDS uint32_t*)(mine + (size_t)p.kf * 8);
  t.ll = (HDA_LDS Ent*)(mine + (size_t)p.kf * 12);
  t.gf = (HDA_GLOBAL Ent*)(p.spill_free + slot * (p.cf - p.kf));
  t.gst = (HDA_GLOBAL uint32_t*)(p.spill_stamp + slot * (p.cf - p.kf));
  t.gl = (HDA_GLOBAL Ent*)(p.spill_live + slot * (p.cl - p.kl));
  t.kf = p.kf; t.kl = p.kl; t.cf = p.cf; t.cl = p.cl;
  if (!p.use_queue) {
    if ((int64_t)slot < p.n_heaps) {
      const int64_t k = p.first + (int64_t)slot;
      replay_one_heap(p, t, p.order ? p.order[k] : k);
    }
    return;
  }
  // A wave can take at most every heap, so the loop is bounded even if the
  // queue were never to run dry.
  for (int64_t taken = 0; taken < p.n_heaps; ++taken) {
    // Every lane takes part in the atomic (lane 0 adds 1, the others 0), so
    // the value read back from lane 0 is not produced under a lane-dependent
    // branch: a wave-wide read of a value written only by some lanes would let
    // the compiler send the other lanes round the loop on their own.
    uint32_t hq = atomicAdd(p.queue, lane_id() == 0 ? 1u : 0u);
    hq = rdlane(hq, 0);
    if ((int64_t)hq >= p.n_heaps) break;
    const int64_t k = p.first + (int64_t)hq;
    replay_one_heap(p, t, p.order ? p.order[k] : k);
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct DeviceInfo {
  int cus = 0;
  size_t max_lds = 0;
};

DeviceInfo device_info() {
  static std::mutex mu;
  static int cached_dev = -1;
  static DeviceInfo cached;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DeviceInfo{};
  std::lock_guard<std::mutex> g(mu);
  if (dev != cached_dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return DeviceInfo{};
    cached.cus = prop.multiProcessorCount;
    cached.max_lds = prop.sharedMemPerBlock;
    if (prop.maxSharedMemoryPerMultiProcessor > cached.max_lds)
      cached.max_lds = prop.maxSharedMemoryPerMultiProcessor;
    cached_dev = dev;
  }
  return cached;
}

uint32_t round64(int64_t x) { return (uint32_t)((x + 63) / 64 * 64); }

struct Plan {
  uint32_t W, kf, kl, cf, cl, lds_wave, lds_group;
  int64_t groups, slots;
  size_t off_queue, off_free, off_stamp, off_live, bytes;
};

// Fill defaults and derive the launch and workspace layout.
bool make_plan(const hda_batch_desc* d, bool persistent, Plan* pl) {
  if (!d || d->n_heaps < 0 || d->meta_free < 0 || d->meta_live < 0) return false;
  const hda_tuning& tu = d->tuning;
  const DeviceInfo di = device_info();
  if (di.cus <= 0) return false;
  uint32_t W = tu.heaps_per_group > 0 ? (uint32_t)tu.heaps_per_group : 4u;
  uint32_t kf = tu.lds_free > 0 ? round64(tu.lds_free) : 256u;
  uint32_t kl = tu.lds_live > 0 ? round64(tu.lds_live) : 768u;
  if (W > 16u || (tu.lds_free % 64) || (tu.lds_live % 64)) return false;
  const uint32_t cf = std::max<uint32_t>(kf, round64(d->meta_free > 0 ? d->meta_free : 4096));
  const uint32_t cl = std::max<uint32_t>(kl, round64(d->meta_live > 0 ? d->meta_live : 8192));
  if (!persistent) W = 1;
  const uint32_t lds_wave = kf * 12u + kl * 8u;
  const uint32_t lds_group = lds_wave * W;
  if (lds_group > di.max_lds || lds_group == 0) return false;
  int64_t groups;
  if (persistent) {
    // resident workgroups per CU as the runtime computes it (LDS, registers,
    // wave slots)
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, replay_kernel, (int)(64 * W),
                                                     (size_t)lds_group) != hipSuccess || nb < 1)
      nb = 1;
    const int64_t per_cu = nb;
    groups = tu.groups > 0 ? tu.groups : per_cu * di.cus;
    const int64_t need = (d->n_heaps + W - 1) / W;
    groups = std::max<int64_t>(1, std::min<int64_t>(groups, need));
  } else {
    groups = 1;
  }
  pl->W = W; pl->kf = kf; pl->kl = kl; pl->cf = cf; pl->cl = cl;
  pl->lds_wave = lds_wave; pl->lds_group = lds_group;
  pl->groups = groups;
  pl->slots = groups * W;
  auto align_up = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t o = 0;
  pl->off_queue = o; o = align_up(o + 4);
  pl->off_free = o; o = align_up(o + (size_t)pl->slots * (cf - kf) * 8);
  pl->off_stamp = o; o = align_up(o + (size_t)pl->slots * (cf - kf) * 4);
  pl->off_live = o; o = align_up(o + (size_t)pl->slots * (cl - kl) * 8);
  pl->bytes = o;
  return true;
}

bool desc_ok(const hda_batch_desc* d) {
  if (!d || d->n_heaps < 0) return false;
  if (d->n_heaps == 0) return true;
  if (!d->arena || !d->align || !d->algo || !d->req_off || !d->req || !d->res || !d->status)
    return false;
  if (d->state && (!d->state_off || !d->state_len)) return false;
  return true;
}

ReplayParams params_from(const hda_batch_desc* d, const Plan& pl) {
  ReplayParams p;
  std::memset(&p, 0, sizeof(p));
  p.arena = d->arena; p.align = d->align; p.algo = d->algo;
  p.req_off = d->req_off; p.req = d->req; p.res = d->res; p.order = d->order;
  p.state = d->state; p.state_off = d->state_off; p.state_len = d->state_len;
  p.status = d->status;
  uint8_t* ws = static_cast<uint8_t*>(d->workspace);
  p.queue = reinterpret_cast<uint32_t*>(ws + pl.off_queue);
  p.spill_free = reinterpret_cast<Ent*>(ws + pl.off_free);
  p.spill_stamp = reinterpret_cast<uint32_t*>(ws + pl.off_stamp);
  p.spill_live = reinterpret_cast<Ent*>(ws + pl.off_live);
  p.n_heaps = d->n_heaps;
  p.first = 0;
  p.kf = pl.kf; p.kl = pl.kl; p.cf = pl.cf; p.cl = pl.cl;
  p.waves_per_group = pl.W;
  p.lds_wave_bytes = pl.lds_wave;
  p.use_queue = 1;
  return p;
}

bool set_lds_attr(uint32_t bytes) {
  static uint32_t done = 0;
  if (bytes <= 65536 || bytes <= done) return true;
  if (hipFuncSetAttribute((const void*)replay_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
    return false;
  done = bytes;
  return true;
}

}  // namespace

extern "C" {

size_t hda_replay_workspace(const hda_batch_desc* d) {
  Plan pl, pl1;
  if (!make_plan(d, true, &pl) || !make_plan(d, false, &pl1)) return 0;
  return std::max(pl.bytes, pl1.bytes);
}

int hda_replay_resolve(const hda_batch_desc* d, hda_tuning* out) {
  Plan pl;
  if (!out || !make_plan(d, true, &pl)) return HDA_E_INVAL;
  out->heaps_per_group = (int32_t)pl.W;
  out->lds_free = (int32_t)pl.kf;
  out->lds_live = (int32_t)pl.kl;
  out->groups = (int32_t)pl.groups;
  return HDA_OK;
}

int hda_replay(const hda_batch_desc* d, void* stream) {
  Plan pl;
  if (!desc_ok(d) || !make_plan(d, true, &pl)) return HDA_E_INVAL;
  if (d->n_heaps == 0) return HDA_OK;
  if (!d->workspace || d->workspace_bytes < pl.bytes) return HDA_E_RANGE;
  ReplayParams p = params_from(d, pl);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!set_lds_attr(pl.lds_group)) return HDA_E_DEVICE;
  hipLaunchKernelGGL(reset_queue, dim3(1), dim3(1), 0, s, p.queue);
  hipLaunchKernelGGL(replay_kernel, dim3((uint32_t)pl.groups), dim3(64 * pl.W),
                     pl.lds_group, s, p);
  return hipGetLastError() == hipSuccess ? HDA_OK : HDA_E_DEVICE;
}

int hda_replay_per_heap(const hda_batch_desc* d, void* stream) {
  Plan pl;
  if (!desc_ok(d) || !make_plan(d, false, &pl)) return HDA_E_INVAL;
  if (d->n_heaps == 0) return HDA_OK;
  if (!d->workspace || d->workspace_bytes < pl.bytes) return HDA_E_RANGE;
  ReplayParams p = params_from(d, pl);
  p.use_queue = 0;
  p.n_heaps = 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!set_lds_attr(pl.lds_group)) return HDA_E_DEVICE;
  for (int64_t k = 0; k < d->n_heaps; ++k) {
    p.first = k;
    hipLaunchKernelGGL(replay_kernel, dim3(1), dim3(64), pl.lds_group, s, p);
  }
  return hipGetLastError() == hipSuccess ? HDA_OK : HDA_E_DEVICE;
}

}  // extern "C"
