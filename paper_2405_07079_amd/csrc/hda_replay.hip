// Batched replay of many independent heaps on gfx950.
//
// A small classify kernel splits the caller's heap order by algorithm (and
// sets heaps with invalid parameters aside, rejecting them); then one
// persistent kernel per algorithm -- compiled for that algorithm alone, so the
// register allocation fits its own tables -- replays its heaps, one wavefront
// per heap, pulling them from a device queue in the caller's order (longest
// trace first is the useful order for uneven batches).  The per-algorithm
// launches run concurrently on library streams forked from and joined back to
// the caller's stream, so a mixed batch finishes when its slowest algorithm
// group does.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "hda.h"
#include "hda_wave.h"
#include "hda_core.h"
#include "hda_replay_body.h"

using namespace hda;

namespace {

constexpr int kClasses = 5;  // four algorithms + invalid

struct ClassifyParams {
  const int64_t* arena;
  const int64_t* align;
  const int32_t* algo;
  const int32_t* order;
  const int64_t* req_off;
  int64_t* res;
  int32_t* status;
  int64_t* state_len;
  int32_t* lists;      // kClasses x n_heaps
  uint32_t* counts;    // kClasses
  uint32_t* queues;    // one per algorithm, cleared here
  int64_t n_heaps;
};

__device__ __forceinline__ bool params_valid(const ClassifyParams& q, int64_t heap) {
  const int64_t A = q.arena[heap], g = q.align[heap];
  const int algo = q.algo[heap];
  return !(algo < 0 || algo > 3 || g <= 0 || (g & (g - 1)) || A <= 0 || (A % g) ||
           (A / g) >= (int64_t(1) << 32));
}

// One workgroup.  Wave 0 compacts `order` into per-class lists keeping the
// order (ballot + popcount below the lane); then every wave rejects a share of
// the invalid heaps.
__global__ void __launch_bounds__(1024) classify_kernel(ClassifyParams q) {
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  __shared__ uint32_t counts[kClasses];
  if (wave == 0) {
    uint32_t cnt[kClasses] = {0, 0, 0, 0, 0};
    const uint64_t below = (1ull << lane) - 1ull;
    for (int64_t base = 0; base < q.n_heaps; base += 64) {
      const int64_t k = base + lane;
      const bool in = k < q.n_heaps;
      const int64_t heap = in ? (q.order ? (int64_t)q.order[k] : k) : 0;
      const int cls = in ? (params_valid(q, heap) ? q.algo[heap] : 4) : kClasses;
#pragma unroll
      for (int a = 0; a < kClasses; ++a) {
        const uint64_t m = ballot(cls == a);
        if (cls == a)
          q.lists[(int64_t)a * q.n_heaps + cnt[a] + __builtin_popcountll(m & below)] = (int32_t)heap;
        cnt[a] += (uint32_t)__builtin_popcountll(m);
      }
    }
    if (lane < (uint32_t)kClasses) {
      uint32_t v = 0;
#pragma unroll
      for (int a = 0; a < kClasses; ++a) v = (lane == (uint32_t)a) ? cnt[a] : v;
      counts[lane] = v;
      q.counts[lane] = v;
      if (lane < 4u) q.queues[lane] = 0u;
    }
  }
  __syncthreads();
  const uint32_t bad = counts[4];
  for (uint32_t i = wave; i < bad; i += waves) {
    const int64_t heap = q.lists[4 * q.n_heaps + i];
    const int64_t b0 = q.req_off[heap], b1 = q.req_off[heap + 1];
    for (int64_t base = b0; base < b1; base += 64)
      if (base + lane < b1) q.res[base + lane] = kEInval;
    if (lane == 0) {
      q.status[heap] = (int32_t)kEInval;
      if (q.state_len) q.state_len[heap] = 0;
    }
  }
}

template <int ALGO, int RF, int RL>
__global__ void __launch_bounds__(1024) replay_kernel(ReplayParams p) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const uint32_t wave = threadIdx.x >> 6;
  HDA_LDS uint8_t* mine = (HDA_LDS uint8_t*)smem + (size_t)wave * p.lds_wave_bytes;
  const uint64_t slot = (uint64_t)blockIdx.x * p.waves_per_group + wave;
  Cold c;
  c.lf = (HDA_LDS Ent*)(mine);
  c.lst = (HDA_LDS uint32_t*)(mine + (size_t)p.kf * 8);
  c.ll = (HDA_LDS Ent*)(mine + (size_t)p.kf * 12);
  c.gf = (HDA_GLOBAL Ent*)(p.spill_free + slot * p.sf);
  c.gst = (HDA_GLOBAL uint32_t*)(p.spill_stamp + slot * p.sf);
  c.gl = (HDA_GLOBAL Ent*)(p.spill_live + slot * p.sl);
  c.kf = p.kf; c.kl = p.kl;
  c.cf = p.kf + p.sf; c.cl = p.kl + p.sl;
  const int64_t n = p.use_queue ? (int64_t)*p.count : p.n_heaps;
  if (!p.use_queue) {
    if ((int64_t)slot < n) replay_one_heap<ALGO, RF, RL>(p, c, p.list[p.first + (int64_t)slot]);
    return;
  }
  // A wave can take at most every heap, so the loop is bounded even if the
  // queue were never to run dry.
  for (int64_t taken = 0; taken < n; ++taken) {
    // Every lane takes part in the atomic (lane 0 adds 1, the others 0), so
    // the value read back from lane 0 is not produced under a lane-dependent
    // branch: a wave-wide read of a value written only by some lanes would let
    // the compiler send the other lanes round the loop on their own.
    uint32_t hq = atomicAdd(p.queue, lane_id() == 0 ? 1u : 0u);
    hq = rdlane(hq, 0);
    if ((int64_t)hq >= n) break;
    replay_one_heap<ALGO, RF, RL>(p, c, p.list[hq]);
  }
}

// Register-resident table shapes the library is compiled for:
// (free chunks, live chunks) of 64 entries each, one kernel per algorithm.
struct Shape {
  int rf, rl;
  const void* fn[4];
};
#define HDA_SHAPE(RF, RL)                                                          \
  {RF, RL, {(const void*)replay_kernel<kFirstFit, RF, RL>,                         \
            (const void*)replay_kernel<kNextFit, RF, RL>,                          \
            (const void*)replay_kernel<kBestFit, RF, RL>,                          \
            (const void*)replay_kernel<kSegFit, RF, RL>}}
const Shape kShapes[] = {HDA_SHAPE(0, 0), HDA_SHAPE(2, 4), HDA_SHAPE(4, 0), HDA_SHAPE(6, 0),
                         HDA_SHAPE(4, 8)};
#undef HDA_SHAPE
constexpr int kDefaultShape = 2;

const Shape* find_shape(int rf, int rl) {
  for (const Shape& s : kShapes)
    if (s.rf == rf && s.rl == rl) return &s;
  return nullptr;
}

struct DeviceCtx {
  int cus = 0;
  size_t max_lds = 0;
  std::mutex enqueue;  // one fork/join sequence at a time on the shared streams
  hipStream_t side[4] = {};
  hipEvent_t fork = nullptr, join[4] = {};
  bool ok = false;
};

// Per-device properties and the library's fork/join streams (default
// priority), created on first use.
DeviceCtx* device_ctx() {
  static std::mutex mu;
  static std::vector<DeviceCtx*> ctxs;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  if ((int)ctxs.size() <= dev) ctxs.resize(dev + 1, nullptr);
  if (!ctxs[dev]) {
    DeviceCtx* c = new DeviceCtx;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      c->cus = prop.multiProcessorCount;
      c->max_lds = std::max<size_t>(prop.sharedMemPerBlock, prop.maxSharedMemoryPerMultiProcessor);
      c->ok = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) == hipSuccess;
      for (int a = 0; a < 4 && c->ok; ++a)
        c->ok = hipStreamCreateWithFlags(&c->side[a], hipStreamNonBlocking) == hipSuccess &&
                hipEventCreateWithFlags(&c->join[a], hipEventDisableTiming) == hipSuccess;
    }
    ctxs[dev] = c;
  }
  return ctxs[dev]->ok ? ctxs[dev] : nullptr;
}

uint32_t round64(int64_t x) { return (uint32_t)((x + 63) / 64 * 64); }

struct Plan {
  const Shape* shape;
  uint32_t W, capF, capL, kf, kl, sf, sl, lds_wave, lds_group;
  int64_t groups[4], slots[4];
  size_t off_counts, off_queues, off_lists, off_free[4], off_stamp[4], off_live[4], bytes;
};

// Fill defaults and derive the launches and the workspace layout.
bool make_plan(const hda_batch_desc* d, bool persistent, Plan* pl) {
  if (!d || d->n_heaps < 0 || d->meta_free < 0 || d->meta_live < 0) return false;
  if (d->n_heaps > INT32_MAX) return false;
  const hda_tuning& tu = d->tuning;
  const DeviceCtx* dc = device_ctx();
  if (!dc) return false;
  // register shape: 0 = default, -1 = none
  const Shape* shape = &kShapes[kDefaultShape];
  if (tu.reg_free != 0 || tu.reg_live != 0) {
    shape = find_shape(tu.reg_free < 0 ? 0 : tu.reg_free, tu.reg_live < 0 ? 0 : tu.reg_live);
    if (!shape) return false;
  }
  if (tu.heaps_per_group < 0 || tu.heaps_per_group > 16 || (tu.lds_free > 0 && tu.lds_free % 64) ||
      (tu.lds_live > 0 && tu.lds_live % 64) || tu.groups < 0)
    return false;
  uint32_t W = tu.heaps_per_group > 0 ? (uint32_t)tu.heaps_per_group : 4u;
  if (!persistent) W = 1;
  const uint32_t capF = round64(d->meta_free > 0 ? d->meta_free : 4096);
  const uint32_t capL = round64(d->meta_live > 0 ? d->meta_live : 8192);
  const uint32_t coldF = capF > 64u * shape->rf ? capF - 64u * shape->rf : 0u;
  const uint32_t coldL = capL > 64u * shape->rl ? capL - 64u * shape->rl : 0u;
  // LDS part of the cold tables: 0 = default, -1 = none
  const uint32_t want_kf = tu.lds_free > 0 ? (uint32_t)tu.lds_free : (tu.lds_free < 0 ? 0u : 64u);
  // default LDS share of the live table: all of it up to 1024 entries when
  // the shape keeps none in registers
  const uint32_t dflt_kl = shape->rl == 0 ? 1024u : 128u;
  const uint32_t want_kl = tu.lds_live > 0 ? (uint32_t)tu.lds_live : (tu.lds_live < 0 ? 0u : dflt_kl);
  const uint32_t kf = std::min(want_kf, coldF), kl = std::min(want_kl, coldL);
  const uint32_t lds_wave = kf * 12u + kl * 8u;
  const uint32_t lds_group = lds_wave * W;
  if (lds_group > dc->max_lds) return false;
  pl->shape = shape;
  pl->W = W; pl->capF = capF; pl->capL = capL;
  pl->kf = kf; pl->kl = kl; pl->sf = coldF - kf; pl->sl = coldL - kl;
  pl->lds_wave = lds_wave; pl->lds_group = lds_group;
  for (int a = 0; a < 4; ++a) {
    int64_t groups = 1;
    if (persistent) {
      // resident workgroups per CU as the runtime computes it (LDS,
      // registers, wave slots)
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, shape->fn[a], (int)(64 * W),
                                                       (size_t)lds_group) != hipSuccess || nb < 1)
        nb = 1;
      groups = tu.groups > 0 ? tu.groups : (int64_t)nb * dc->cus;
      const int64_t need = (d->n_heaps + W - 1) / W;
      groups = std::max<int64_t>(1, std::min<int64_t>(groups, need));
    }
    pl->groups[a] = groups;
    pl->slots[a] = groups * W;
  }
  auto align_up = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t o = 0;
  pl->off_counts = o; o = align_up(o + kClasses * 4);
  pl->off_queues = o; o = align_up(o + 4 * 4);
  pl->off_lists = o; o = align_up(o + (size_t)kClasses * std::max<int64_t>(d->n_heaps, 1) * 4);
  for (int a = 0; a < 4; ++a) {
    pl->off_free[a] = o; o = align_up(o + (size_t)pl->slots[a] * pl->sf * 8);
    pl->off_stamp[a] = o; o = align_up(o + (size_t)pl->slots[a] * pl->sf * 4);
    pl->off_live[a] = o; o = align_up(o + (size_t)pl->slots[a] * pl->sl * 8);
  }
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

ClassifyParams classify_params(const hda_batch_desc* d, const Plan& pl) {
  ClassifyParams q;
  uint8_t* ws = static_cast<uint8_t*>(d->workspace);
  q.arena = d->arena; q.align = d->align; q.algo = d->algo; q.order = d->order;
  q.req_off = d->req_off; q.res = d->res; q.status = d->status; q.state_len = d->state_len;
  q.lists = reinterpret_cast<int32_t*>(ws + pl.off_lists);
  q.counts = reinterpret_cast<uint32_t*>(ws + pl.off_counts);
  q.queues = reinterpret_cast<uint32_t*>(ws + pl.off_queues);
  q.n_heaps = d->n_heaps;
  return q;
}

ReplayParams replay_params(const hda_batch_desc* d, const Plan& pl, int a) {
  ReplayParams p;
  std::memset(&p, 0, sizeof(p));
  p.arena = d->arena; p.align = d->align; p.algo = d->algo;
  p.req_off = d->req_off; p.req = d->req; p.res = d->res; p.order = d->order;
  p.state = d->state; p.state_off = d->state_off; p.state_len = d->state_len;
  p.status = d->status;
  uint8_t* ws = static_cast<uint8_t*>(d->workspace);
  p.list = reinterpret_cast<const int32_t*>(ws + pl.off_lists) + (int64_t)a * d->n_heaps;
  p.count = reinterpret_cast<const uint32_t*>(ws + pl.off_counts) + a;
  p.queue = reinterpret_cast<uint32_t*>(ws + pl.off_queues) + a;
  p.spill_free = reinterpret_cast<Ent*>(ws + pl.off_free[a]);
  p.spill_stamp = reinterpret_cast<uint32_t*>(ws + pl.off_stamp[a]);
  p.spill_live = reinterpret_cast<Ent*>(ws + pl.off_live[a]);
  p.n_heaps = d->n_heaps;
  p.first = 0;
  p.cap_free = pl.capF; p.cap_live = pl.capL;
  p.kf = pl.kf; p.kl = pl.kl; p.sf = pl.sf; p.sl = pl.sl;
  p.waves_per_group = pl.W;
  p.lds_wave_bytes = pl.lds_wave;
  p.use_queue = 1;
  return p;
}

bool set_lds_attr(const Shape* s, uint32_t bytes) {
  if (bytes <= 65536) return true;
  for (int a = 0; a < 4; ++a)
    if (hipFuncSetAttribute(s->fn[a], hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) !=
        hipSuccess)
      return false;
  return true;
}

hipError_t launch(const void* fn, dim3 grid, dim3 block, uint32_t lds, hipStream_t st,
                  ReplayParams& p) {
  void* args[] = {&p};
  return hipLaunchKernel(fn, grid, block, args, lds, st);
}

int classify(const hda_batch_desc* d, const Plan& pl, hipStream_t s) {
  ClassifyParams q = classify_params(d, pl);
  hipLaunchKernelGGL(classify_kernel, dim3(1), dim3(1024), 0, s, q);
  return hipGetLastError() == hipSuccess ? HDA_OK : HDA_E_DEVICE;
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
  out->reg_free = pl.shape->rf > 0 ? pl.shape->rf : -1;
  out->reg_live = pl.shape->rl > 0 ? pl.shape->rl : -1;
  out->lds_free = pl.kf > 0 ? (int32_t)pl.kf : -1;
  out->lds_live = pl.kl > 0 ? (int32_t)pl.kl : -1;
  out->groups = (int32_t)pl.groups[0];
  return HDA_OK;
}

int hda_replay(const hda_batch_desc* d, void* stream) {
  Plan pl;
  if (!desc_ok(d) || !make_plan(d, true, &pl)) return HDA_E_INVAL;
  if (d->n_heaps == 0) return HDA_OK;
  if (!d->workspace || d->workspace_bytes < pl.bytes) return HDA_E_RANGE;
  DeviceCtx* dc = device_ctx();
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!dc || !set_lds_attr(pl.shape, pl.lds_group)) return HDA_E_DEVICE;
  std::lock_guard<std::mutex> g(dc->enqueue);
  int rc = classify(d, pl, s);
  if (rc != HDA_OK) return rc;
  if (hipEventRecord(dc->fork, s) != hipSuccess) return HDA_E_DEVICE;
  for (int a = 0; a < 4; ++a) {
    ReplayParams p = replay_params(d, pl, a);
    if (hipStreamWaitEvent(dc->side[a], dc->fork, 0) != hipSuccess ||
        launch(pl.shape->fn[a], dim3((uint32_t)pl.groups[a]), dim3(64 * pl.W), pl.lds_group,
               dc->side[a], p) != hipSuccess ||
        hipEventRecord(dc->join[a], dc->side[a]) != hipSuccess ||
        hipStreamWaitEvent(s, dc->join[a], 0) != hipSuccess)
      return HDA_E_DEVICE;
  }
  return hipGetLastError() == hipSuccess ? HDA_OK : HDA_E_DEVICE;
}

int hda_replay_per_heap(const hda_batch_desc* d, void* stream) {
  Plan pl;
  if (!desc_ok(d) || !make_plan(d, false, &pl)) return HDA_E_INVAL;
  if (d->n_heaps == 0) return HDA_OK;
  if (!d->workspace || d->workspace_bytes < pl.bytes) return HDA_E_RANGE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!set_lds_attr(pl.shape, pl.lds_group)) return HDA_E_DEVICE;
  int rc = classify(d, pl, s);
  if (rc != HDA_OK) return rc;
  // the host needs each heap's algorithm to pick the kernel it launches
  uint32_t counts[kClasses];
  const uint8_t* ws = static_cast<const uint8_t*>(d->workspace);
  if (hipMemcpyAsync(counts, ws + pl.off_counts, sizeof(counts), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return HDA_E_DEVICE;
  for (int a = 0; a < 4; ++a) {
    ReplayParams p = replay_params(d, pl, a);
    p.use_queue = 0;
    p.n_heaps = 1;
    for (uint32_t k = 0; k < counts[a]; ++k) {
      p.first = k;
      if (launch(pl.shape->fn[a], dim3(1), dim3(64), pl.lds_group, s, p) != hipSuccess)
        return HDA_E_DEVICE;
    }
  }
  return hipGetLastError() == hipSuccess ? HDA_OK : HDA_E_DEVICE;
}

}  // extern "C"
