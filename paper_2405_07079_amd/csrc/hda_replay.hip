// Batched replay of many independent heaps on gfx950.
//
// A small classify kernel keeps the heaps with valid parameters in the
// caller's order (rejecting the others); then one persistent kernel replays
// them, one wavefront per heap, each wave pulling the next heap from a device
// queue.  The kernel holds all four algorithms and switches per heap, so a
// mixed batch is taken in one order (longest trace first is the useful order
// for uneven batches) instead of one algorithm after another.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "hda.h"
#include "hda_wave.h"
#include "hda_core.h"
#include "hda_replay_body.h"
#include "hda_ordered.h"
#include "hda_mem.h"

using namespace hda;

namespace {

constexpr int kClasses = 2;  // heaps with valid parameters, and the others
constexpr int kValid = 0, kInvalid = 1;
// Queue words in the workspace: the heap queue, the number of heaps moved
// from the lean to the general core, and the queue of the ordered-core launch.
constexpr int kQueueWords = 3;
constexpr int kMigrated = 1;
constexpr int kHeavyQueue = 2;

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
  return !(algo < 0 || algo > kTlsf || g <= 0 || (g & (g - 1)) || A <= 0 || (A % g) ||
           (A / g) >= (int64_t(1) << 32));
}

// One workgroup.  Wave 0 compacts `order` into the lists of valid and invalid
// heaps keeping the order (ballot + popcount below the lane); then every wave
// rejects a share of the invalid heaps.
__global__ void __launch_bounds__(1024) classify_kernel(ClassifyParams q) {
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  __shared__ uint32_t counts[kClasses];
  if (wave == 0) {
    uint32_t cnt[kClasses] = {0, 0};
    const uint64_t below = (1ull << lane) - 1ull;
    for (int64_t base = 0; base < q.n_heaps; base += 64) {
      const int64_t k = base + lane;
      const bool in = k < q.n_heaps;
      const int64_t heap = in ? (q.order ? (int64_t)q.order[k] : k) : 0;
      const int cls = in ? (params_valid(q, heap) ? kValid : kInvalid) : kClasses;
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
    }
    if (lane < (uint32_t)kQueueWords) q.queues[lane] = 0u;
  }
  __syncthreads();
  const uint32_t bad = counts[kInvalid];
  for (uint32_t i = wave; i < bad; i += waves) {
    const int64_t heap = q.lists[kInvalid * q.n_heaps + i];
    const int64_t b0 = q.req_off[heap], b1 = q.req_off[heap + 1];
    for (int64_t base = b0; base < b1; base += 64)
      if (base + lane < b1) q.res[base + lane] = kEInval;
    if (lane == 0) {
      q.status[heap] = (int32_t)kEInval;
      if (q.state_len) q.state_len[heap] = 0;
    }
  }
}

// Persistent loop: waves pull list positions list_lo, list_lo + 1, ... from
// p.queue until min(list_hi, the list's length) is reached; with use_queue =
// 0 wave `slot` takes list entry first + slot.
template <typename Fn>
__device__ __forceinline__ void for_each_heap(const ReplayParams& p, uint64_t slot, Fn&& f) {
  if (!p.use_queue) {
    if ((int64_t)slot < p.n_heaps) f((int64_t)p.list[p.first + (int64_t)slot]);
    return;
  }
  const int64_t len = (int64_t)*p.count;
  const int64_t hi = len < p.list_hi ? len : p.list_hi;
  const int64_t n = hi - p.list_lo;
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
    f((int64_t)p.list[p.list_lo + (int64_t)hq]);
  }
}

// General path: tables in LDS, then device memory (per wave slot).
__device__ __forceinline__ Cold general_tiers(const ReplayParams& p, HDA_LDS uint8_t* mine,
                                              uint64_t slot) {
  Cold c;
  c.lf = (HDA_LDS Ent*)(mine);
  c.lst = (HDA_LDS uint32_t*)(mine + (size_t)p.kf * 8);
  c.ll = (HDA_LDS Ent*)(mine + (size_t)p.kf * 12);
  c.gf = (HDA_GLOBAL Ent*)(p.spill_free + slot * p.sf);
  c.gst = (HDA_GLOBAL uint32_t*)(p.spill_stamp + slot * p.sf);
  c.gl = (HDA_GLOBAL Ent*)(p.spill_live + slot * p.sl);
  c.kf = p.kf; c.kl = p.kl;
  c.cf = p.kf + p.sf; c.cl = p.kl + p.sl;
  return c;
}

// General path for every heap (tables in LDS, then device memory).
__global__ void __launch_bounds__(1024) general_kernel(ReplayParams p) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const uint32_t wave = uniform(threadIdx.x >> 6);  // the same in every lane of the wave
  HDA_LDS uint8_t* mine = (HDA_LDS uint8_t*)smem + (size_t)wave * p.lds_wave_bytes;
  const uint64_t slot = (uint64_t)blockIdx.x * p.waves_per_group + wave;
  const Cold c = general_tiers(p, mine, slot);
  for_each_heap(p, slot, [&](int64_t heap) __attribute__((always_inline)) {
    replay_any_heap<0, 0>(p, c, heap);
  });
}

// Lean path with RF free-table chunks in VGPRs; each heap runs the code of
// its own algorithm.
template <int RF>
__global__ void __launch_bounds__(1024) lean_kernel(ReplayParams p) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const uint32_t wave = uniform(threadIdx.x >> 6);  // the same in every lane of the wave
  HDA_LDS uint8_t* mine = (HDA_LDS uint8_t*)smem + (size_t)wave * p.lds_wave_bytes;
  const uint64_t slot = (uint64_t)blockIdx.x * p.waves_per_group + wave;
  LeanLds lds;
  lds.base = mine;
  lds.bytes = p.lds_wave_bytes;
  // the general core's tiers for a heap that outgrows the pool: this wave's
  // device-memory slot (no LDS part)
  const Cold c = general_tiers(p, mine, slot);
  for_each_heap(p, slot, [&](int64_t heap) __attribute__((always_inline)) {
    switch (p.algo[heap]) {
      case kFirstFit: lean_one_heap<kFirstFit, RF>(p, lds, c, heap); break;
      case kNextFit: lean_one_heap<kNextFit, RF>(p, lds, c, heap); break;
      case kBestFit: lean_one_heap<kBestFit, RF>(p, lds, c, heap); break;
      case kSegFit: lean_one_heap<kSegFit, RF>(p, lds, c, heap); break;
      case kTlsf: lean_one_heap<kTlsf, RF>(p, lds, c, heap); break;
      default: reject_heap(p, heap); break;  // the bitmask allocator has its own kernel
    }
  });
}

// Ordered core (hda_ordered.h) for the heaps taken first from the order: one
// wave per workgroup owning the whole dynamic LDS of the launch as its pool,
// and a device-memory slot per workgroup for what does not fit.
__global__ void __launch_bounds__(64) ordered_kernel(ReplayParams p) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  HDA_LDS uint8_t* pool = (HDA_LDS uint8_t*)smem;
  const uint64_t slot = blockIdx.x;
  HDA_GLOBAL uint8_t* dev = (HDA_GLOBAL uint8_t*)(p.ord_dev + slot * p.ord_dev_stride);
  for_each_heap(p, slot, [&](int64_t heap) __attribute__((always_inline)) {
    ord_any_heap(p, pool, dev, heap);
  });
}

// Kernels by free-table chunks in VGPRs (0 = general path).
struct KernelSet {
  int rf;
  const void* fn;
};
const KernelSet kSets[] = {{0, (const void*)general_kernel},
                           {1, (const void*)lean_kernel<1>},
                           {2, (const void*)lean_kernel<2>},
                           {4, (const void*)lean_kernel<4>}};
constexpr int kDefaultRF = 2;

const KernelSet* find_set(int rf) {
  for (const KernelSet& s : kSets)
    if (s.rf == rf) return &s;
  return nullptr;
}

struct DeviceCtx {
  int cus = 0;
  size_t max_lds = 0;
  bool ok = false;
};

// Per-device properties, read on first use.
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
      c->ok = true;
    }
    ctxs[dev] = c;
  }
  return ctxs[dev]->ok ? ctxs[dev] : nullptr;
}

uint32_t round64(int64_t x) { return (uint32_t)((x + 63) / 64 * 64); }

// Launch geometry and tiers of the replay kernel.
struct Pass {
  uint32_t W = 1, kf = 0, kl = 0, sf = 0, sl = 0, lds_wave = 0, lds_group = 0;
  uint32_t lds_free = 0, lds_live = 0;  // the LDS residency as the tuning states it
  int64_t groups = 1, slots = 1;
  size_t off_free = 0, off_stamp = 0, off_live = 0;
};

struct Plan {
  const KernelSet* set;
  bool lean;
  uint32_t capF, capL;
  Pass main;
  // the ordered-core launch: the first `heavy` heaps of the order, one wave
  // per workgroup with a pool of heavy_pool LDS bytes, heavy_groups of them
  int64_t heavy = 0;
  uint32_t heavy_pool = 0, heavy_slot_bytes = 0;
  int64_t heavy_groups = 0;
  uint64_t heavy_stride = 0;
  size_t off_ord = 0;
  size_t off_counts, off_queues, off_lists, bytes;
};

int occupancy_groups(const void* fn, uint32_t W, uint32_t lds_group, int cus, int32_t want,
                     int64_t n_heaps) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, (int)(64 * W), (size_t)lds_group) !=
          hipSuccess ||
      nb < 1)
    nb = 1;
  int64_t groups = want > 0 ? want : (int64_t)nb * cus;
  const int64_t need = (n_heaps + W - 1) / W;
  return (int)std::max<int64_t>(1, std::min<int64_t>(groups, need));
}

// Fill defaults and derive the launches and the workspace layout.
bool make_plan(const hda_batch_desc* d, bool persistent, Plan* pl) {
  if (!d || d->n_heaps < 0 || d->meta_free < 0 || d->meta_live < 0) return false;
  if (d->n_heaps > INT32_MAX) return false;
  const hda_tuning& tu = d->tuning;
  const DeviceCtx* dc = device_ctx();
  if (!dc) return false;
  // free chunks in registers: 0 = default, -1 = none (general path); the
  // live table is never held in registers
  const int rf = tu.reg_free == 0 ? kDefaultRF : (tu.reg_free < 0 ? 0 : tu.reg_free);
  const KernelSet* set = find_set(rf);
  if (!set || tu.reg_live > 0) return false;
  if (tu.heaps_per_group < 0 || tu.heaps_per_group > 16 || (tu.lds_free > 0 && tu.lds_free % 64) ||
      (tu.lds_live > 0 && tu.lds_live % 64) || tu.groups < 0 || tu.heavy_heaps < 0 ||
      tu.heavy_kib < 0)
    return false;
  const bool lean = rf > 0;
  uint32_t W = tu.heaps_per_group > 0 ? (uint32_t)tu.heaps_per_group : 4u;
  if (!persistent) W = 1;
  const uint32_t capF = round64(d->meta_free > 0 ? d->meta_free : 4096);
  const uint32_t capL = round64(d->meta_live > 0 ? d->meta_live : 8192);
  // LDS entries: 0 = default, -1 = none
  const uint32_t want_kf = tu.lds_free > 0 ? (uint32_t)tu.lds_free
                                           : (tu.lds_free < 0 ? 0u : (lean ? 128u : 64u));
  // (lean: the pool, lds_free * 16 + lds_live * 8 bytes; general: LDS tiers)
  const uint32_t want_kl = tu.lds_live > 0 ? (uint32_t)tu.lds_live : (tu.lds_live < 0 ? 0u : 1024u);
  Pass& m = pl->main;
  m.W = W;
  if (lean) {
    // one LDS pool per wave with room for want_kf segregated-fit free
    // entries (16 B) and want_kl live entries (8 B); a heap that outgrows it
    // continues on the general core in its device-memory slot
    m.kf = m.kl = 0;
    m.sf = capF;
    m.sl = capL;
    m.lds_wave = (want_kf * 16u + want_kl * 8u + 15u) & ~15u;
    m.lds_free = want_kf;
    m.lds_live = want_kl;
  } else {
    // LDS parts never exceed the capacities; entries past them are in device
    // memory
    m.kf = std::min(want_kf, capF);
    m.kl = std::min(want_kl, capL);
    m.sf = capF - m.kf;
    m.sl = capL - m.kl;
    m.lds_wave = m.kf * 12u + m.kl * 8u;
    m.lds_free = m.kf;
    m.lds_live = m.kl;
  }
  m.lds_group = m.lds_wave * W;
  if (m.lds_group > dc->max_lds) return false;
  // the ordered-core launch (persistent replays only)
  const int64_t heavy = persistent ? std::min<int64_t>(tu.heavy_heaps, d->n_heaps) : 0;
  int heavy_cus = 0;
  if (heavy > 0) {
    const uint32_t kib = tu.heavy_kib > 0 ? (uint32_t)tu.heavy_kib : 64u;
    if (kib < 16u || (size_t)kib * 1024u > dc->max_lds) return false;
    if (capF > kOrdMaxFree) return false;  // the ordered core holds at most this many
    pl->heavy = heavy;
    pl->heavy_pool = kib * 1024u;
    // TLSF's list heads first, then half of the rest for chunk slots
    pl->heavy_slot_bytes = (pl->heavy_pool - kOrdTlsfHeadBytes) / 2u;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)ordered_kernel, 64,
                                                     (size_t)pl->heavy_pool) != hipSuccess ||
        nb < 1)
      nb = 1;
    pl->heavy_groups = std::max<int64_t>(1, std::min<int64_t>(heavy, (int64_t)nb * dc->cus));
    heavy_cus = (int)((pl->heavy_groups + nb - 1) / nb);
    pl->heavy_stride = (ord_dev_bytes(capL) + 255) / 256 * 256;
  }
  // the other heaps fill the CUs the ordered-core launch leaves
  const int light_cus = std::max(1, dc->cus - heavy_cus);
  m.groups = persistent ? occupancy_groups(set->fn, W, m.lds_group, light_cus, tu.groups,
                                           d->n_heaps - heavy)
                        : 1;
  m.slots = m.groups * W;
  pl->set = set;
  pl->lean = lean;
  pl->capF = capF;
  pl->capL = capL;
  auto align_up = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t off = 0;
  pl->off_counts = off; off = align_up(off + kClasses * 4);
  pl->off_queues = off; off = align_up(off + kQueueWords * 4);
  const size_t H1 = (size_t)std::max<int64_t>(d->n_heaps, 1);
  pl->off_lists = off; off = align_up(off + (size_t)kClasses * H1 * 4);
  m.off_free = off; off = align_up(off + (size_t)m.slots * m.sf * 8);
  m.off_stamp = off; off = align_up(off + (size_t)m.slots * m.sf * 4);
  m.off_live = off; off = align_up(off + (size_t)m.slots * m.sl * 8);
  pl->off_ord = off; off = align_up(off + (size_t)pl->heavy_groups * pl->heavy_stride);
  pl->bytes = off;
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

// Parameters of the replay launch.
ReplayParams replay_params(const hda_batch_desc* d, const Plan& pl) {
  const Pass& ps = pl.main;
  ReplayParams p;
  std::memset(&p, 0, sizeof(p));
  p.arena = d->arena; p.align = d->align; p.algo = d->algo;
  p.req_off = d->req_off; p.req = d->req; p.res = d->res; p.order = d->order;
  p.state = d->state; p.state_off = d->state_off; p.state_len = d->state_len;
  p.status = d->status;
  uint8_t* ws = static_cast<uint8_t*>(d->workspace);
  uint32_t* queues = reinterpret_cast<uint32_t*>(ws + pl.off_queues);
  p.list = reinterpret_cast<const int32_t*>(ws + pl.off_lists) + (int64_t)kValid * d->n_heaps;
  p.count = reinterpret_cast<const uint32_t*>(ws + pl.off_counts) + kValid;
  p.queue = queues;
  p.migrated = queues + kMigrated;
  p.spill_free = reinterpret_cast<Ent*>(ws + ps.off_free);
  p.spill_stamp = reinterpret_cast<uint32_t*>(ws + ps.off_stamp);
  p.spill_live = reinterpret_cast<Ent*>(ws + ps.off_live);
  p.n_heaps = d->n_heaps;
  p.first = 0;
  p.cap_free = pl.capF; p.cap_live = pl.capL;
  p.kf = ps.kf; p.kl = ps.kl; p.sf = ps.sf; p.sl = ps.sl;
  p.waves_per_group = ps.W;
  p.lds_wave_bytes = ps.lds_wave;
  p.use_queue = 1;
  p.list_lo = pl.heavy;
  p.list_hi = INT64_MAX;
  return p;
}

// Parameters of the ordered-core launch: list positions [0, heavy), its own
// queue counter, its device slots.
ReplayParams heavy_params(const hda_batch_desc* d, const Plan& pl) {
  ReplayParams p = replay_params(d, pl);
  uint8_t* ws = static_cast<uint8_t*>(d->workspace);
  p.queue = reinterpret_cast<uint32_t*>(ws + pl.off_queues) + kHeavyQueue;
  p.list_lo = 0;
  p.list_hi = pl.heavy;
  p.ord_pool_bytes = pl.heavy_pool;
  p.ord_slot_bytes = pl.heavy_slot_bytes;
  p.ord_dev = ws + pl.off_ord;
  p.ord_dev_stride = pl.heavy_stride;
  return p;
}

bool set_lds_attr(const void* fn, uint32_t bytes) {
  if (bytes <= 65536) return true;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
         hipSuccess;
}

bool set_lds_attrs(const Plan& pl) {
  return set_lds_attr(pl.set->fn, pl.main.lds_group) &&
         (pl.heavy == 0 || set_lds_attr((const void*)ordered_kernel, pl.heavy_pool));
}

// A second stream per device for the launch that runs beside the
// ordered-core one (default priority, not blocking the null stream).
hipStream_t fork_stream() {
  static std::mutex mu;
  static std::vector<hipStream_t> streams;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
  if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
    streams[dev] = nullptr;
  return streams[dev];
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

// Classify, then the persistent replay kernel, both on s.  With heaps for
// the ordered core, their launch follows classify on s and the other heaps'
// launch runs beside it on the fork stream, joined back to s by an event.
int enqueue(const hda_batch_desc* d, const Plan& pl, hipStream_t s) {
  int rc = classify(d, pl, s);
  if (rc != HDA_OK) return rc;
  ReplayParams p = replay_params(d, pl);
  const dim3 grid((uint32_t)pl.main.groups), block(64 * pl.main.W);
  if (pl.heavy == 0) {
    if (launch(pl.set->fn, grid, block, pl.main.lds_group, s, p) != hipSuccess)
      return HDA_E_DEVICE;
    return hipGetLastError() == hipSuccess ? HDA_OK : HDA_E_DEVICE;
  }
  hipStream_t f = fork_stream();
  if (!f) return HDA_E_DEVICE;
  hipEvent_t e_fork = nullptr, e_join = nullptr;
  rc = HDA_E_DEVICE;
  ReplayParams hp = heavy_params(d, pl);
  if (hipEventCreateWithFlags(&e_fork, hipEventDisableTiming) == hipSuccess &&
      hipEventCreateWithFlags(&e_join, hipEventDisableTiming) == hipSuccess &&
      hipEventRecord(e_fork, s) == hipSuccess &&
      launch((const void*)ordered_kernel, dim3((uint32_t)pl.heavy_groups), dim3(64),
             pl.heavy_pool, s, hp) == hipSuccess &&
      hipStreamWaitEvent(f, e_fork, 0) == hipSuccess &&
      launch(pl.set->fn, grid, block, pl.main.lds_group, f, p) == hipSuccess &&
      hipEventRecord(e_join, f) == hipSuccess && hipStreamWaitEvent(s, e_join, 0) == hipSuccess)
    rc = hipGetLastError() == hipSuccess ? HDA_OK : HDA_E_DEVICE;
  if (e_fork) (void)hipEventDestroy(e_fork);
  if (e_join) (void)hipEventDestroy(e_join);
  return rc;
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
  out->heaps_per_group = (int32_t)pl.main.W;
  out->reg_free = pl.set->rf > 0 ? pl.set->rf : -1;
  out->reg_live = -1;
  out->lds_free = pl.main.lds_free > 0 ? (int32_t)pl.main.lds_free : -1;
  out->lds_live = pl.main.lds_live > 0 ? (int32_t)pl.main.lds_live : -1;
  out->groups = (int32_t)pl.main.groups;
  out->heavy_heaps = (int32_t)pl.heavy;
  out->heavy_kib = pl.heavy > 0 ? (int32_t)(pl.heavy_pool / 1024u) : 0;
  return HDA_OK;
}

int hda_replay(const hda_batch_desc* d, void* stream) {
  Plan pl;
  if (!desc_ok(d) || !make_plan(d, true, &pl)) return HDA_E_INVAL;
  if (d->n_heaps == 0) return HDA_OK;
  if (!d->workspace || d->workspace_bytes < pl.bytes) return HDA_E_RANGE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!set_lds_attrs(pl)) return HDA_E_DEVICE;
  return enqueue(d, pl, s);
}

int hda_replay_per_heap(const hda_batch_desc* d, void* stream) {
  Plan pl;
  if (!desc_ok(d) || !make_plan(d, false, &pl)) return HDA_E_INVAL;
  if (d->n_heaps == 0) return HDA_OK;
  if (!d->workspace || d->workspace_bytes < pl.bytes) return HDA_E_RANGE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!set_lds_attrs(pl)) return HDA_E_DEVICE;
  int rc = classify(d, pl, s);
  if (rc != HDA_OK) return rc;
  // the host needs the number of valid heaps to launch one kernel per heap
  uint32_t counts[kClasses];
  const uint8_t* ws = static_cast<const uint8_t*>(d->workspace);
  if (hipMemcpyAsync(counts, ws + pl.off_counts, sizeof(counts), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return HDA_E_DEVICE;
  ReplayParams p = replay_params(d, pl);
  p.use_queue = 0;
  p.n_heaps = 1;
  for (uint32_t k = 0; k < counts[kValid]; ++k) {
    p.first = k;
    if (launch(pl.set->fn, dim3(1), dim3(64), pl.main.lds_group, s, p) != hipSuccess)
      return HDA_E_DEVICE;
  }
  return hipGetLastError() == hipSuccess ? HDA_OK : HDA_E_DEVICE;
}

// The longest heaps (by trace length), longest first: at most `want` of them
// and, past `min_heaps`, no more than `budget` requests once each trace is cut
// to `cut` requests.
static std::vector<int32_t> longest_heaps(const std::vector<int64_t>& off, int64_t want,
                                          int64_t min_heaps, int64_t budget, int64_t cut) {
  const int64_t H = (int64_t)off.size() - 1;
  std::vector<int32_t> idx(H);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
    return off[a + 1] - off[a] > off[b + 1] - off[b];
  });
  std::vector<int32_t> out;
  int64_t total = 0;
  for (int64_t k = 0; k < H && k < want; ++k) {
    const int64_t len = std::min(off[idx[k] + 1] - off[idx[k]], cut);
    if (k >= min_heaps && total + len > budget) break;
    total += len;
    out.push_back(idx[k]);
  }
  return out;
}

}  // extern "C"

namespace {

// Time each candidate tuning on a private batch made of the heaps in
// `sample` (indices into the caller's batch), each trace cut to `cut`
// requests, in that order (one untimed trial first).  *pick receives the
// fastest candidate.
int time_candidates(const hda_batch_desc* d, const std::vector<int64_t>& off,
                    const std::vector<int64_t>& arena, const std::vector<int64_t>& align,
                    const std::vector<int32_t>& algo, const std::vector<int32_t>& sample,
                    int64_t cut, const std::vector<hda_tuning>& cand, hipStream_t s,
                    hda_tuning* pick) {
  const int64_t S = (int64_t)sample.size();
  std::vector<int64_t> s_off(S + 1, 0), s_arena(S), s_align(S);
  std::vector<int32_t> s_algo(S);
  for (int64_t k = 0; k < S; ++k) {
    const int32_t h = sample[k];
    s_off[k + 1] = s_off[k] + std::min(off[h + 1] - off[h], cut);
    s_arena[k] = arena[h];
    s_align[k] = align[h];
    s_algo[k] = algo[h];
  }
  const int64_t N = std::max<int64_t>(s_off[S], 1);
  // the trial batch: its own buffers, so the caller's outputs are untouched
  hda_batch_desc dd;
  std::memset(&dd, 0, sizeof(dd));
  dd.n_heaps = S;
  dd.meta_free = d->meta_free;
  dd.meta_live = d->meta_live;
  size_t ws = 0;
  std::vector<hda_tuning> ok;
  for (const hda_tuning& t : cand) {
    dd.tuning = t;
    Plan p2;
    if (make_plan(&dd, true, &p2)) {
      ok.push_back(t);
      ws = std::max(ws, p2.bytes);
    }
  }
  if (ok.empty()) return HDA_E_INVAL;
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t o_arena = 0, o_align = up(o_arena + S * 8), o_algo = up(o_align + S * 8),
               o_off = up(o_algo + S * 4), o_req = up(o_off + (S + 1) * 8),
               o_res = up(o_req + N * 8), o_status = up(o_res + N * 8),
               o_work = up(o_status + S * 4), bytes = o_work + ws;
  uint8_t* buf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = HDA_E_DEVICE;
  float best = -1.0f;
  *pick = ok[0];
  buf = static_cast<uint8_t*>(dev_alloc(bytes));
  if (buf && hipEventCreate(&e0) == hipSuccess &&
      hipEventCreate(&e1) == hipSuccess &&
      hipMemcpyAsync(buf + o_arena, s_arena.data(), S * 8, hipMemcpyHostToDevice, s) ==
          hipSuccess &&
      hipMemcpyAsync(buf + o_align, s_align.data(), S * 8, hipMemcpyHostToDevice, s) ==
          hipSuccess &&
      hipMemcpyAsync(buf + o_algo, s_algo.data(), S * 4, hipMemcpyHostToDevice, s) ==
          hipSuccess &&
      hipMemcpyAsync(buf + o_off, s_off.data(), (S + 1) * 8, hipMemcpyHostToDevice, s) ==
          hipSuccess) {
    rc = HDA_OK;
    for (int64_t k = 0; k < S && rc == HDA_OK; ++k) {
      const size_t n = (size_t)(s_off[k + 1] - s_off[k]);
      if (n && hipMemcpyAsync(buf + o_req + s_off[k] * 8, d->req + off[sample[k]], n * 8,
                              hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = HDA_E_DEVICE;
    }
    dd.arena = reinterpret_cast<const int64_t*>(buf + o_arena);
    dd.align = reinterpret_cast<const int64_t*>(buf + o_align);
    dd.algo = reinterpret_cast<const int32_t*>(buf + o_algo);
    dd.req_off = reinterpret_cast<const int64_t*>(buf + o_off);
    dd.req = reinterpret_cast<const int64_t*>(buf + o_req);
    dd.res = reinterpret_cast<int64_t*>(buf + o_res);
    dd.status = reinterpret_cast<int32_t*>(buf + o_status);
    dd.workspace = buf + o_work;
    dd.workspace_bytes = ws;
    // one untimed trial first (code objects, LDS attributes), then one each
    for (size_t i = 0; i <= ok.size() && rc == HDA_OK; ++i) {
      dd.tuning = ok[i == 0 ? 0 : i - 1];
      if (hipEventRecord(e0, s) != hipSuccess || hda_replay(&dd, s) != HDA_OK ||
          hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = HDA_E_DEVICE;
        break;
      }
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = HDA_E_DEVICE;
      if (i > 0 && (best < 0.0f || ms < best)) {
        best = ms;
        *pick = ok[i - 1];
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (buf) {
    (void)hipStreamSynchronize(s);
    dev_free(buf);
  }
  return rc;
}

// Choices of earlier autotuner calls, keyed by the device and the batch's
// shape (heap count, capacities, sample size, the caller's register tier,
// and a hash of every heap's trace length, arena, alignment and algorithm):
// a batch of the same shape on the same device reuses the choice without
// timing again.  Any choice gives the same results.
struct TuneKey {
  int dev;
  int64_t heaps, meta_free, meta_live;
  int32_t sample, reg_free;
  uint64_t shape;
  bool operator==(const TuneKey& o) const {
    return dev == o.dev && heaps == o.heaps && meta_free == o.meta_free &&
           meta_live == o.meta_live && sample == o.sample && reg_free == o.reg_free &&
           shape == o.shape;
  }
};
constexpr size_t kTuneCacheMax = 64;  // shapes remembered; the oldest goes first
std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, hda_tuning>> g_tune_cache;

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {  // FNV-1a, 64 bits
  const uint8_t* b = static_cast<const uint8_t*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 0x100000001b3ull;
  return h;
}

}  // namespace

extern "C" {

int hda_replay_autotune(const hda_batch_desc* d, int32_t sample_heaps, void* stream,
                        hda_tuning* out) {
  constexpr int64_t kCut = 65536, kBudget = int64_t(16) << 20;
  constexpr int64_t kHeavyCut = int64_t(1) << 20;
  Plan pl;
  if (!out || !desc_ok(d) || sample_heaps < 0 || !make_plan(d, true, &pl)) return HDA_E_INVAL;
  DeviceCtx* dc = device_ctx();
  if (!dc) return HDA_E_DEVICE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t H = d->n_heaps;
  if (H == 0) return hda_replay_resolve(d, out);
  // heap parameters and trace lengths on the host
  std::vector<int64_t> off(H + 1), arena(H), align(H);
  std::vector<int32_t> algo(H);
  if (hipMemcpyAsync(off.data(), d->req_off, off.size() * 8, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(arena.data(), d->arena, H * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(align.data(), d->align, H * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(algo.data(), d->algo, H * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return HDA_E_DEVICE;
  TuneKey key{0, H, d->meta_free, d->meta_live, sample_heaps, d->tuning.reg_free, 0xcbf29ce484222325ull};
  if (hipGetDevice(&key.dev) != hipSuccess) return HDA_E_DEVICE;
  for (int64_t h = 0; h < H; ++h) {
    const int64_t len = off[h + 1] - off[h];
    key.shape = fnv1a(key.shape, &len, 8);
    key.shape = fnv1a(key.shape, &arena[h], 8);
    key.shape = fnv1a(key.shape, &align[h], 8);
    key.shape = fnv1a(key.shape, &algo[h], 4);
  }
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (const auto& e : g_tune_cache)
      if (e.first == key) {
        hda_batch_desc dp = *d;
        dp.tuning = e.second;
        return hda_replay_resolve(&dp, out);
      }
  }
  // 1. heaps per workgroup and the lean path's LDS residency, on the longest
  // heaps, as many as the device holds at once under the default tuning,
  // each trace cut to its first kCut requests
  const int64_t want = sample_heaps > 0 ? sample_heaps : pl.main.slots;
  const std::vector<int32_t> sample = longest_heaps(off, want, dc->cus, kBudget, kCut);
  std::vector<hda_tuning> cand;
  const uint32_t lds_pairs[][2] = {{64, 512}, {128, 1024}, {256, 2048}, {512, 4096}};
  for (int32_t W : {1, 2, 4, 8, 16})
    for (const auto& kv : lds_pairs) {
      hda_tuning t = d->tuning;
      t.heaps_per_group = W;
      t.reg_free = t.reg_free < 0 ? 0 : t.reg_free;
      t.reg_live = 0;
      t.lds_free = (int32_t)kv[0];
      t.lds_live = (int32_t)kv[1];
      t.groups = 0;
      t.heavy_heaps = 0;
      t.heavy_kib = 0;
      cand.push_back(t);
    }
  hda_tuning pick;
  int rc = time_candidates(d, off, arena, align, algo, sample, kCut, cand, s, &pick);
  if (rc == HDA_E_INVAL) return hda_replay_resolve(d, out);
  if (rc != HDA_OK) return rc;
  // 2. how many of the longest heaps the ordered core takes (0, 16, 64,
  // 128, or every sampled heap when fewer), timed on the 128 longest heaps
  // with traces up to kHeavyCut requests, so that their tables reach the
  // sizes that set the makespan.  The ordered core holds at most
  // kOrdMaxFree free blocks: with larger meta_free it is not tried.
  if (d->meta_free <= (int64_t)kOrdMaxFree) {
    const std::vector<int32_t> longest = longest_heaps(off, 128, 1, kBudget, kHeavyCut);
    const int64_t S2 = (int64_t)longest.size();
    std::vector<hda_tuning> hc;
    hda_tuning t = pick;
    hc.push_back(t);
    for (int64_t k : {int64_t(16), int64_t(64), int64_t(128)}) {
      if (k > S2 && (k != 16 || S2 == 0)) continue;
      t.heavy_heaps = (int32_t)std::min<int64_t>(k, S2);
      t.heavy_kib = 64;
      hc.push_back(t);
    }
    if (hc.size() > 1) {
      hda_tuning pick2;
      rc = time_candidates(d, off, arena, align, algo, longest, kHeavyCut, hc, s, &pick2);
      if (rc != HDA_OK && rc != HDA_E_INVAL) return rc;
      if (rc == HDA_OK) pick = pick2;
    }
  }
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (g_tune_cache.size() >= kTuneCacheMax) g_tune_cache.erase(g_tune_cache.begin());
    g_tune_cache.push_back({key, pick});
  }
  hda_batch_desc dp = *d;
  dp.tuning = pick;
  return hda_replay_resolve(&dp, out);
}

}  // extern "C"

// ---- replay without allocation ----
//
// The device scratch of hda_replay_static: one array per GPU the library
// runs on, held until the process ends.  Its name is a host-side stand-in in
// host code; kernels are only ever given the device address that
// hipGetSymbolAddress returns for the current device.
namespace {
constexpr size_t kStaticScratchBytes = size_t(HDA_STATIC_SCRATCH_BYTES);
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

// The scratch's device address on the current device, looked up once per
// device (with that device current); nullptr if the lookup fails.
uint8_t* static_scratch() {
  static std::mutex mu;
  static std::vector<uint8_t*> ptrs;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  if ((int)ptrs.size() <= dev) ptrs.resize(dev + 1, nullptr);
  if (!ptrs[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    ptrs[dev] = static_cast<uint8_t*>(ptr);
  }
  return ptrs[dev];
}
}  // namespace

extern "C" {

int hda_replay_static(const hda_batch_desc* d, void* stream) {
  Plan pl;
  if (!desc_ok(d) || !make_plan(d, true, &pl)) return HDA_E_INVAL;
  if (pl.heavy > 0) return HDA_E_INVAL;  // events and a second stream: use hda_replay
  if (d->n_heaps == 0) return HDA_OK;
  if (pl.bytes > kStaticScratchBytes) return HDA_E_RANGE;
  uint8_t* ws = static_scratch();
  if (!ws) return HDA_E_DEVICE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!set_lds_attrs(pl)) return HDA_E_DEVICE;
  // the same launches as hda_replay, with the scratch as their workspace;
  // the classify kernel clears the queue counters (no memset), and every
  // spill entry is written before it is read
  hda_batch_desc dd = *d;
  dd.workspace = ws;
  dd.workspace_bytes = kStaticScratchBytes;
  return enqueue(&dd, pl, s);
}

}  // extern "C"

struct hda_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

int hda_replay_capture(const hda_batch_desc* d, hda_graph** out) {
  Plan pl;
  if (!out || !desc_ok(d) || !make_plan(d, true, &pl) || d->n_heaps == 0) return HDA_E_INVAL;
  if (!d->workspace || d->workspace_bytes < pl.bytes) return HDA_E_RANGE;
  if (!set_lds_attrs(pl)) return HDA_E_DEVICE;
  if (pl.heavy > 0 && !fork_stream()) return HDA_E_DEVICE;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return HDA_E_DEVICE;
  hda_graph* g = new hda_graph;
  int rc = HDA_E_DEVICE;
  {
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      const int erc = enqueue(d, pl, cs);
      const hipError_t ec = hipStreamEndCapture(cs, &g->graph);
      if (erc == HDA_OK && ec == hipSuccess &&
          hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) == hipSuccess)
        rc = HDA_OK;
      else if (erc != HDA_OK)
        rc = erc;
    }
  }
  (void)hipStreamDestroy(cs);
  if (rc != HDA_OK) {
    hda_graph_destroy(g);
    return rc;
  }
  *out = g;
  return HDA_OK;
}

int hda_graph_launch(hda_graph* g, void* stream) {
  if (!g || !g->exec) return HDA_E_INVAL;
  return hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? HDA_OK
                                                                               : HDA_E_DEVICE;
}

int hda_graph_destroy(hda_graph* g) {
  if (!g) return HDA_E_INVAL;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return HDA_OK;
}

}  // extern "C"
