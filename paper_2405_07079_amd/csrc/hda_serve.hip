// Device-resident allocator service with continuous batching.
//
// Every admitted heap keeps its registers and tables in a slot of a device
// memory pool.  A persistent kernel of `waves` wavefronts serves them: heap
// slot s belongs to wave s % waves, which polls its own submission ring (in
// pinned, coherent host memory), applies the requests in order with the same
// allocator code as the call-by-call heaps (Alg. 1-5), and publishes each
// result in its completion ring.  Requests of different heaps run on
// different waves at the same time, and a request submitted while others are
// in flight is taken by its wave as soon as the wave gets to it.
//
// Exit: a wave leaves its loop when the host raises the stop flag or when the
// watchdog (max_seconds of the device wall clock) expires, so every wave ends
// even if the host process never stops it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "hda.h"
#include "hda_wave.h"
#include "hda_core.h"
#include "hda_heap_dev.h"
#include "hda_mem.h"

using namespace hda;

namespace {

enum : int32_t { kSrvInit = 3, kSrvClose = 4 };  // beside HDA_OP_ALLOC / HDA_OP_FREE

struct SubEntry {
  int32_t slot;
  int32_t op;
  int64_t arg;
  int64_t arg2;
  uint64_t seq;
};
// A completion: the result, the request's sequence number and three device
// wall-clock readings -- when the wave first saw the request in its ring,
// when it began serving it, and when it had served it.
struct CplEntry {
  int64_t result;
  uint64_t seq;
  uint64_t t_seen, t_pick, t_done;
  uint64_t pad[3];
};
// Per wave: this header, then SubEntry[N], then CplEntry[N].
struct RingHdr {
  uint64_t sub_tail;   // requests submitted (written by the host)
  uint64_t pad0[15];
  uint64_t cpl_tail;   // requests completed (written by the device)
  uint64_t pad1[15];
};

struct ServeParams {
  uint8_t* rings;
  uint64_t ring_bytes;
  uint32_t N;
  int32_t waves;
  uint8_t* pool;
  uint64_t slot_bytes;
  int32_t max_heaps;
  uint32_t cf, cl;
  uint32_t* stop;
  uint64_t max_ticks;
};

__device__ __forceinline__ uint64_t rdlane64(uint64_t v, uint32_t l) {
  return ((uint64_t)rdlane((uint32_t)(v >> 32), l) << 32) | rdlane((uint32_t)v, l);
}

__device__ __forceinline__ Cold slot_cold(uint8_t* slot, uint32_t cf, uint32_t cl) {
  uint8_t* base = slot + sizeof(HeapHdr);
  Cold c;
  c.lf = nullptr; c.lst = nullptr; c.ll = nullptr;
  c.kf = 0; c.kl = 0;
  c.cf = cf; c.cl = cl;
  c.gf = (HDA_GLOBAL Ent*)(base);
  c.gst = (HDA_GLOBAL uint32_t*)(base + (size_t)cf * 8);
  c.gl = (HDA_GLOBAL Ent*)(base + (size_t)cf * 12);
  return c;
}

template <int ALGO>
__device__ int64_t run_op(uint8_t* slot, const ServeParams& p, const HeapRegs& regs, int op,
                          int64_t arg) {
  HeapHdr* hd = reinterpret_cast<HeapHdr*>(slot);
  WaveHeap<ALGO, 0, 0> w(slot_cold(slot, p.cf, p.cl), regs, p.cf, p.cl);
  int64_t r = 0;
  if (op == kSrvInit) w.init();
  else if (op == HDA_OP_ALLOC) r = arg < 0 ? kEInval : w.alloc_bytes(arg);
  else r = w.free_offset(arg);
  store_regs(hd, w.h);
  return r;
}

__device__ int64_t serve_one(const ServeParams& p, int32_t slot_id, int op, int64_t arg,
                             int64_t arg2) {
  if (slot_id < 0 || slot_id >= p.max_heaps) return kEInval;
  uint8_t* slot = p.pool + (uint64_t)slot_id * p.slot_bytes;
  HeapHdr* hd = reinterpret_cast<HeapHdr*>(slot);
  HeapRegs h;
  if (op == kSrvInit) {
    // arg = arena bytes, arg2 = algo << 8 | log2(align); validated by the host
    h.algo = (int)(arg2 >> 8);
    h.shift = (uint32_t)(arg2 & 255);
    h.arena = arg;
    h.ag = (uint32_t)((uint64_t)arg >> h.shift);
    h.status = 0;
    h.F = h.L = h.rover = h.clock = h.cnt = 0;
    if (lane_id() == 0) {
      hd->algo = h.algo; hd->shift = h.shift; hd->arena = h.arena; hd->ag = h.ag;
      hd->cf = p.cf; hd->cl = p.cl;
    }
  } else if (op == HDA_OP_ALLOC || op == HDA_OP_FREE) {
    h = load_regs(hd);
  } else {
    return 0;  // close: nothing on the device
  }
  switch (h.algo) {
    case kFirstFit: return run_op<kFirstFit>(slot, p, h, op, arg);
    case kNextFit: return run_op<kNextFit>(slot, p, h, op, arg);
    case kBestFit: return run_op<kBestFit>(slot, p, h, op, arg);
    case kSegFit: return run_op<kSegFit>(slot, p, h, op, arg);
    default: return run_op<kTlsf>(slot, p, h, op, arg);
  }
}

__global__ void __launch_bounds__(256) serve_kernel(ServeParams p) {
  const int32_t wave = (int32_t)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (wave >= p.waves) return;
  uint8_t* ring = p.rings + (uint64_t)wave * p.ring_bytes;
  RingHdr* hdr = reinterpret_cast<RingHdr*>(ring);
  SubEntry* sub = reinterpret_cast<SubEntry*>(ring + sizeof(RingHdr));
  CplEntry* cpl = reinterpret_cast<CplEntry*>(ring + sizeof(RingHdr) + (uint64_t)p.N * sizeof(SubEntry));
  const uint64_t mask = p.N - 1u;
  const uint64_t t0 = rdlane64(wall_clock64(), 0);
  uint64_t head = 0;
  for (;;) {
    // every value that decides control flow is taken from lane 0
    const uint64_t now = rdlane64(wall_clock64(), 0);
    if (now - t0 > p.max_ticks) break;
    uint64_t tail = __hip_atomic_load(&hdr->sub_tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
    tail = rdlane64(tail, 0);
    if (tail == head) {
      uint32_t stop = __hip_atomic_load(p.stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
      stop = rdlane(stop, 0);
      if (stop != 0u) break;
      __builtin_amdgcn_s_sleep(8);
      continue;
    }
    // never more than a ring's worth per pass; every request of the pass was
    // seen at `seen`
    const uint64_t end = tail - head > p.N ? head + p.N : tail;
    const uint64_t seen = now;
    for (; head < end; ++head) {
      const uint64_t t_pick = rdlane64(wall_clock64(), 0);
      // one 32-byte read of the entry: lanes 0..3 fetch its four words
      const uint64_t* e = reinterpret_cast<const uint64_t*>(&sub[head & mask]);
      const uint64_t word = e[lane_id() & 3u];
      const uint64_t w0 = rdlane64(word, 0);
      const int32_t slot = (int32_t)(uint32_t)w0;
      const int32_t op = (int32_t)(uint32_t)(w0 >> 32);
      const int64_t arg = (int64_t)rdlane64(word, 1);
      const int64_t arg2 = (int64_t)rdlane64(word, 2);
      const uint64_t seq = rdlane64(word, 3);
      const int64_t r = serve_one(p, slot, op, arg, arg2);
      const uint64_t t_done = rdlane64(wall_clock64(), 0);
      if (lane_id() == 0) {
        cpl[head & mask].result = r;
        cpl[head & mask].seq = seq;
        cpl[head & mask].t_seen = seen;
        cpl[head & mask].t_pick = t_pick;
        cpl[head & mask].t_done = t_done;
        __hip_atomic_store(&hdr->cpl_tail, head + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct RingState {
  std::mutex mu;
  uint64_t tail = 0;        // submitted
  uint64_t harvested = 0;   // completions copied out
  std::vector<int64_t> results;
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct hda_server {
  hda_serve_config cfg{};
  int device = 0;
  int G = 0;
  uint32_t N = 0;
  uint64_t ring_bytes = 0;
  uint8_t* rings = nullptr;
  uint32_t* stop = nullptr;
  uint8_t* pool = nullptr;
  uint64_t slot_bytes = 0;
  uint32_t cf = 0, cl = 0;
  hipStream_t stream = nullptr;
  std::unique_ptr<RingState[]> rs;
  std::mutex slots_mu;
  std::vector<int32_t> free_slots;  // descending: back() is the smallest
  int64_t held = 0, budget = 0;
  bool running = false;

  RingHdr* hdr(int r) { return reinterpret_cast<RingHdr*>(rings + (uint64_t)r * ring_bytes); }
  SubEntry* sub(int r) { return reinterpret_cast<SubEntry*>(rings + (uint64_t)r * ring_bytes + sizeof(RingHdr)); }
  CplEntry* cpl(int r) {
    return reinterpret_cast<CplEntry*>(rings + (uint64_t)r * ring_bytes + sizeof(RingHdr) +
                                       (uint64_t)N * sizeof(SubEntry));
  }
  // copy new completions of ring r (caller holds rs[r].mu)
  void harvest(int r) {
    RingState& s = rs[r];
    const uint64_t ct = __atomic_load_n(&hdr(r)->cpl_tail, __ATOMIC_ACQUIRE);
    CplEntry* c = cpl(r);
    for (uint64_t q = s.harvested; q < ct; ++q) s.results[q & (N - 1)] = c[q & (N - 1)].result;
    if (ct > s.harvested) s.harvested = ct;
  }
  // enqueue one entry on the ring of `slot`; returns the ticket.  With
  // may_harvest false (the load generator, which consumes completions
  // itself) a full ring returns kFullRing instead of waiting.
  static constexpr uint64_t kFullRing = ~0ull;
  uint64_t push(int32_t slot, int32_t op, int64_t arg, int64_t arg2, bool may_harvest = true) {
    const int r = slot % G;
    RingState& s = rs[r];
    std::unique_lock<std::mutex> g(s.mu);
    while (s.tail - s.harvested >= N) {
      if (!may_harvest) return kFullRing;
      harvest(r);
      if (s.tail - s.harvested >= N) {
        g.unlock();
        std::this_thread::yield();
        g.lock();
      }
    }
    SubEntry* e = &sub(r)[s.tail & (N - 1)];
    e->slot = slot; e->op = op; e->arg = arg; e->arg2 = arg2; e->seq = s.tail;
    const uint64_t t = s.tail++;
    __atomic_store_n(&hdr(r)->sub_tail, s.tail, __ATOMIC_RELEASE);
    return ((uint64_t)r << 40) | t;
  }
  int poll(uint64_t ticket, int64_t* result, int* done) {
    const int r = (int)(ticket >> 40);
    const uint64_t q = ticket & ((1ull << 40) - 1);
    if (r < 0 || r >= G) return HDA_E_INVAL;
    RingState& s = rs[r];
    std::lock_guard<std::mutex> g(s.mu);
    harvest(r);
    if (q >= s.tail) return HDA_E_INVAL;
    if (q >= s.harvested) { *done = 0; return HDA_OK; }
    if (s.harvested - q > N) return HDA_E_RANGE;
    *result = s.results[q & (N - 1)];
    *done = 1;
    return HDA_OK;
  }
};

namespace {

// Wait for a ticket; gives up (HDA_E_BUSY) after 30 s without a completion,
// e.g. when the service kernel has already stopped.
int wait_ticket(hda_server* s, uint64_t t, int64_t* result) {
  const double give_up = now_s() + 30.0;
  for (;;) {
    int done = 0;
    const int rc = s->poll(t, result, &done);
    if (rc != HDA_OK) return rc;
    if (done) return HDA_OK;
    if (now_s() > give_up) return HDA_E_BUSY;
    std::this_thread::yield();
  }
}

bool arena_ok(uint64_t arena, uint64_t align, int algo) {
  return algo >= HDA_FIRST_FIT && algo <= HDA_TLSF && align != 0 && !(align & (align - 1)) &&
         arena != 0 && arena % align == 0 && arena <= (uint64_t)INT64_MAX &&
         arena / align < (uint64_t(1) << 32);
}

}  // namespace

extern "C" {

int hda_serve_start(const hda_serve_config* cfg, hda_server** out) {
  if (!cfg || !out) return HDA_E_INVAL;
  *out = nullptr;
  hda_serve_config c = *cfg;
  if (c.max_heaps <= 0 || c.waves < 0 || c.slot_free < 0 || c.slot_live < 0 ||
      c.ring_entries < 0 || c.meta_budget < 0 || c.max_seconds < 0)
    return HDA_E_INVAL;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return HDA_E_DEVICE;
  if (c.waves == 0) c.waves = 2 * prop.multiProcessorCount;
  if (c.slot_free == 0) c.slot_free = 512;
  if (c.slot_live == 0) c.slot_live = 512;
  if (c.ring_entries == 0) c.ring_entries = 1024;
  if (c.max_seconds == 0) c.max_seconds = 600;
  if (c.ring_entries & (c.ring_entries - 1)) return HDA_E_INVAL;
  std::unique_ptr<hda_server> s(new (std::nothrow) hda_server);
  if (!s) return HDA_E_DEVICE;
  s->cfg = c;
  s->device = dev;
  s->G = c.waves;
  s->N = (uint32_t)c.ring_entries;
  s->cf = (uint32_t)((c.slot_free + 63) / 64 * 64);
  s->cl = (uint32_t)((c.slot_live + 63) / 64 * 64);
  s->slot_bytes = (heap_bytes(s->cf, s->cl) + 255) / 256 * 256;
  s->ring_bytes = (sizeof(RingHdr) + (uint64_t)s->N * (sizeof(SubEntry) + sizeof(CplEntry)) + 255) / 256 * 256;
  s->budget = c.meta_budget > 0 ? c.meta_budget : (int64_t)s->slot_bytes * c.max_heaps;
  s->rs.reset(new RingState[s->G]);
  for (int r = 0; r < s->G; ++r) s->rs[r].results.assign(s->N, 0);
  for (int32_t k = c.max_heaps - 1; k >= 0; --k) s->free_slots.push_back(k);
  const size_t ring_total = s->ring_bytes * (size_t)s->G;
  if (hipHostMalloc((void**)&s->rings, ring_total, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
      hipHostMalloc((void**)&s->stop, 256, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
      !(s->pool = static_cast<uint8_t*>(dev_alloc(s->slot_bytes * (size_t)c.max_heaps))) ||
      hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
    if (s->rings) (void)hipHostFree(s->rings);
    if (s->stop) (void)hipHostFree(s->stop);
    dev_free(s->pool);
    return HDA_E_DEVICE;
  }
  std::memset(s->rings, 0, ring_total);
  std::memset(s->stop, 0, 256);
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;
  uint8_t* drings = nullptr;
  uint32_t* dstop = nullptr;
  if (hipHostGetDevicePointer((void**)&drings, s->rings, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&dstop, s->stop, 0) != hipSuccess)
    return HDA_E_DEVICE;
  ServeParams p;
  p.rings = drings;
  p.ring_bytes = s->ring_bytes;
  p.N = s->N;
  p.waves = s->G;
  p.pool = s->pool;
  p.slot_bytes = s->slot_bytes;
  p.max_heaps = c.max_heaps;
  p.cf = s->cf; p.cl = s->cl;
  p.stop = dstop;
  p.max_ticks = (uint64_t)(c.max_seconds * 1000.0 * khz);
  const int per_block = 4;
  hipLaunchKernelGGL(serve_kernel, dim3((s->G + per_block - 1) / per_block), dim3(64 * per_block),
                     0, s->stream, p);
  if (hipGetLastError() != hipSuccess) return HDA_E_DEVICE;
  s->running = true;
  *out = s.release();
  return HDA_OK;
}

int hda_serve_open(hda_server* s, uint64_t arena, uint64_t align, int algo, int32_t* heap) {
  if (!s || !heap || !arena_ok(arena, align, algo)) return HDA_E_INVAL;
  int32_t slot;
  {
    std::lock_guard<std::mutex> g(s->slots_mu);
    if (s->free_slots.empty() || s->held + (int64_t)s->slot_bytes > s->budget) return HDA_E_NOMETA;
    slot = s->free_slots.back();
    s->free_slots.pop_back();
    s->held += (int64_t)s->slot_bytes;
  }
  const int64_t arg2 = ((int64_t)algo << 8) | (int64_t)__builtin_ctzll(align);
  s->push(slot, kSrvInit, (int64_t)arena, arg2);
  *heap = slot;
  return HDA_OK;
}

int hda_serve_submit(hda_server* s, int32_t heap, int op, int64_t arg, uint64_t* ticket) {
  if (!s || !ticket || heap < 0 || heap >= s->cfg.max_heaps ||
      (op != HDA_OP_ALLOC && op != HDA_OP_FREE))
    return HDA_E_INVAL;
  *ticket = s->push(heap, op, arg, 0);
  return HDA_OK;
}

int hda_serve_poll(hda_server* s, uint64_t ticket, int64_t* result, int* done) {
  if (!s || !result || !done) return HDA_E_INVAL;
  return s->poll(ticket, result, done);
}

int hda_serve_wait(hda_server* s, uint64_t ticket, int64_t* result) {
  if (!s || !result) return HDA_E_INVAL;
  return wait_ticket(s, ticket, result);
}

int hda_serve_close(hda_server* s, int32_t heap) {
  if (!s || heap < 0 || heap >= s->cfg.max_heaps) return HDA_E_INVAL;
  int64_t r = 0;
  const int rc = wait_ticket(s, s->push(heap, kSrvClose, 0, 0), &r);
  if (rc != HDA_OK) return rc;
  std::lock_guard<std::mutex> g(s->slots_mu);
  s->free_slots.push_back(heap);
  s->held -= (int64_t)s->slot_bytes;
  return HDA_OK;
}

int hda_serve_stop(hda_server* s) {
  if (!s) return HDA_E_INVAL;
  __atomic_store_n(s->stop, 1u, __ATOMIC_RELEASE);
  const hipError_t e = hipStreamSynchronize(s->stream);
  (void)hipStreamDestroy(s->stream);
  dev_free(s->pool);
  (void)hipHostFree(s->rings);
  (void)hipHostFree(s->stop);
  delete s;
  return e == hipSuccess ? HDA_OK : HDA_E_DEVICE;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Open-loop load generator
// ---------------------------------------------------------------------------

namespace {

struct Rng {  // SplitMix64 (Steele, Lea, Flood 2014)
  uint64_t x;
  uint64_t next() {
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

struct Client {
  int32_t heap = -1;                   // -1: no heap (waiting for admission)
  Rng rng{0};
  int64_t t = 0;                       // requests issued
  bool busy = false;
  int op = 0;
  int64_t arg = 0, life = 0, issued_at = 0;
  double arrival = 0, submitted = 0;
  uint64_t arena = 0;                  // the client's arena bytes
  int64_t session_left = 0;            // requests left in this session (sessions)
  std::deque<double> waiting;
  std::vector<std::pair<int64_t, int64_t>> live;  // min-heap on expiry: (expiry, offset)
};

struct LoadShared {
  const hda_load_config* cfg;
  hda_server* s;
  std::vector<Client>* clients;
  double t_warm, t_end;
  double us_per_tick;   // device wall clock
  std::atomic<int64_t> open_now{0}, open_max{0};
};

struct ThreadOut {
  std::vector<float> lat_us;
  // components of each measured latency: waiting on the host before the
  // submission, device queueing (seen -> picked), device service (picked ->
  // done), and the rest (ring transit both ways and the host's harvest)
  std::vector<float> host_us, queue_us, service_us, transit_us;
  int64_t issued = 0, completed = 0, measured = 0, in_window = 0;
  int64_t alloc_ok = 0, alloc_fail = 0, frees = 0, errors = 0;
  int64_t sessions = 0, admission_waits = 0;
};

uint64_t log_uniform(Rng& r, double lo, double hi) {
  double v = std::floor(std::exp(std::log(lo) + r.uniform() * std::log(hi / lo)));
  return (uint64_t)std::min(std::max(v, lo), hi);
}

// Enqueue on a ring that only this load thread consumes.  Each client has at
// most an initialisation and one request or close in flight, and a ring
// serves fewer than half as many clients as it has entries, so a full ring
// frees up as the device works; a ring still full after 10 s (the service
// gone) gives kFullRing, which the caller counts as an error.
uint64_t push_load(hda_server* s, int32_t slot, int32_t op, int64_t arg, int64_t arg2) {
  uint64_t t = s->push(slot, op, arg, arg2, false);
  const double give_up = now_s() + 10.0;
  while (t == hda_server::kFullRing && now_s() < give_up) {
    std::this_thread::yield();
    t = s->push(slot, op, arg, arg2, false);
  }
  return t;
}

// owner marks in a ring position: >= 0 a client's request, -1 nothing of
// the load's, <= -2 the close of client -(mark + 2)'s heap
constexpr int32_t kNoOwner = -1;
int32_t close_mark(int32_t cid) { return -2 - cid; }

void note_open(LoadShared& L, int64_t d) {
  const int64_t n = L.open_now.fetch_add(d) + d;
  int64_t m = L.open_max.load();
  while (n > m && !L.open_max.compare_exchange_weak(m, n)) {
  }
}

// Admit a heap for client c whose ring belongs to load thread p of T (so the
// thread that consumes that ring also owns the client), within the metadata
// budget: the slot closest to the end of the free list among those of the
// thread's rings.  Queues the heap's initialisation.  False when the budget
// or the thread's slots are used up.
bool open_for_thread(LoadShared& L, Client& c, int32_t cid, int p, int T) {
  hda_server* s = L.s;
  const hda_load_config& cfg = *L.cfg;
  int32_t slot = -1;
  {
    std::lock_guard<std::mutex> g(s->slots_mu);
    if (s->held + (int64_t)s->slot_bytes > s->budget) return false;
    for (size_t k = s->free_slots.size(); k-- > 0;) {
      const int32_t cand = s->free_slots[k];
      if ((cand % s->G) % T == p) {
        slot = cand;
        s->free_slots.erase(s->free_slots.begin() + (ptrdiff_t)k);
        break;
      }
    }
    if (slot < 0) return false;
    s->held += (int64_t)s->slot_bytes;
  }
  const int64_t arg2 = ((int64_t)cfg.algo << 8) | (int64_t)__builtin_ctzll(cfg.align);
  if (push_load(s, slot, kSrvInit, (int64_t)c.arena, arg2) == hda_server::kFullRing) {
    std::lock_guard<std::mutex> g(s->slots_mu);
    s->free_slots.push_back(slot);
    s->held -= (int64_t)s->slot_bytes;
    return false;
  }
  c.heap = slot;
  c.session_left = cfg.session_len;
  c.live.clear();
  note_open(L, 1);
  if (cid < cfg.log_clients && cfg.log && cfg.log_len) {  // a session starts: (0, arena, align)
    const int64_t n = cfg.log_len[cid];
    if (n < cfg.log_cap) {
      int64_t* e = cfg.log + ((int64_t)cid * cfg.log_cap + n) * 3;
      e[0] = 0; e[1] = (int64_t)c.arena; e[2] = (int64_t)cfg.align;
      cfg.log_len[cid] = n + 1;
    }
  }
  return true;
}

// Issue client c's next request (arrived at `arrival`); false if it could
// not be enqueued (the client is then left idle).
bool issue(LoadShared& L, Client& c, int32_t cid, double arrival,
           std::vector<int32_t>& owner_of) {
  const hda_load_config& cfg = *L.cfg;
  auto cmp = [](const std::pair<int64_t, int64_t>& a, const std::pair<int64_t, int64_t>& b) {
    return a.first > b.first;
  };
  if (!c.live.empty() && c.live.front().first <= c.t) {
    std::pop_heap(c.live.begin(), c.live.end(), cmp);
    c.arg = c.live.back().second;
    c.live.pop_back();
    c.op = HDA_OP_FREE;
  } else {
    uint64_t size;
    if (c.rng.uniform() < cfg.p_pow2) {
      const int k = cfg.pow2_lo + (int)(c.rng.uniform() * (cfg.pow2_hi - cfg.pow2_lo + 1));
      size = 1ull << std::min(k, cfg.pow2_hi);
    } else {
      size = log_uniform(c.rng, (double)cfg.size_lo, (double)cfg.size_hi);
    }
    c.arg = (int64_t)size;
    c.op = HDA_OP_ALLOC;
    c.life = (int64_t)std::ceil(-cfg.lifetime_mean * std::log(1.0 - c.rng.uniform()));
    if (c.life < 1) c.life = 1;
  }
  c.issued_at = c.t++;
  c.arrival = arrival;
  c.submitted = now_s();
  c.busy = true;
  if (cfg.session_len > 0) --c.session_left;
  const uint64_t ticket = push_load(L.s, c.heap, c.op, c.arg, 0);
  if (ticket == hda_server::kFullRing) return false;
  owner_of[(ticket >> 40) * L.s->N + (ticket & (L.s->N - 1))] = cid;
  return true;
}

void run_thread(LoadShared& L, int p, int T, ThreadOut& out) {
  hda_server* s = L.s;
  const hda_load_config& cfg = *L.cfg;
  std::vector<Client>& cl = *L.clients;
  // this thread's rings are r = p, p+T, ...; its clients are those whose heap
  // lives on them (and, with sessions, those waiting for admission whose
  // number is p mod T).  Only this thread submits to or consumes those rings.
  std::vector<int> rings;
  for (int r = p; r < s->G; r += T) rings.push_back(r);
  std::vector<int32_t> mine;
  std::deque<int32_t> pending;  // clients waiting for admission, first come first
  for (int32_t c = 0; c < (int32_t)cl.size(); ++c) {
    const bool ours = cl[c].heap >= 0 ? (cl[c].heap % s->G) % T == p : c % T == p;
    if (!ours) continue;
    mine.push_back(c);
    if (cl[c].heap < 0) pending.push_back(c);
  }
  // owner_of: completion slot -> client (or a close mark), for every ring
  std::vector<int32_t> owner(s->G * (size_t)s->N, kNoOwner);
  Rng arr{cfg.seed * 0x9e3779b97f4a7c15ull + (uint64_t)p * 7919 + 1};
  const double rate = cfg.rate / T;
  double next = now_s();
  const double t_warm = L.t_warm, t_end = L.t_end;
  if (mine.empty()) return;
  // room for every latency this thread can record (the offered rate's share
  // over the window, with margin), so that no vector grows -- a reallocation
  // would copy hundreds of megabytes while requests wait
  const size_t expect = (size_t)(cfg.rate / T * (t_end - t_warm) * 1.3) + 4096;
  for (std::vector<float>* v : {&out.lat_us, &out.host_us, &out.queue_us, &out.service_us,
                                &out.transit_us})
    v->reserve(expect);
  std::vector<uint64_t> seen(rings.size(), 0);
  for (size_t k = 0; k < rings.size(); ++k) {
    std::lock_guard<std::mutex> g(s->rs[rings[k]].mu);
    seen[k] = s->rs[rings[k]].harvested;
  }
  auto cmp = [](const std::pair<int64_t, int64_t>& a, const std::pair<int64_t, int64_t>& b) {
    return a.first > b.first;
  };
  int64_t busy = 0;      // requests and closes in flight
  for (;;) {
    const double now = now_s();
    bool did = false;
    // admit waiting clients while the budget allows, in arrival order
    while (!pending.empty()) {
      const int32_t cid = pending.front();
      Client& c = cl[cid];
      if (!open_for_thread(L, c, cid, p, T)) break;
      pending.pop_front();
      did = true;
      if (!c.waiting.empty()) {
        const double a = c.waiting.front();
        c.waiting.pop_front();
        if (issue(L, c, cid, a, owner)) {
          ++busy;
          ++out.issued;
        } else {
          c.busy = false;
          ++out.errors;
        }
      }
    }
    while (next <= now && next < t_end) {
      const int32_t cid = mine[(size_t)(arr.uniform() * mine.size()) % mine.size()];
      Client& c = cl[cid];
      if (c.busy || c.heap < 0) {
        if (c.heap < 0 && !c.busy && c.waiting.empty()) ++out.admission_waits;
        c.waiting.push_back(next);
      } else {
        if (issue(L, c, cid, next, owner)) {
          ++busy;
          ++out.issued;
        } else {
          c.busy = false;
          ++out.errors;
        }
      }
      next += -std::log(1.0 - arr.uniform()) / rate;
      did = true;
    }
    for (size_t k = 0; k < rings.size(); ++k) {
      const int r = rings[k];
      const uint64_t ct = __atomic_load_n(&s->hdr(r)->cpl_tail, __ATOMIC_ACQUIRE);
      if (ct == seen[k]) continue;
      const double tc = now_s();
      CplEntry* ce = s->cpl(r);
      for (uint64_t q = seen[k]; q < ct; ++q) {
        const int64_t res = ce[q & (s->N - 1)].result;
        const int32_t who = owner[(size_t)r * s->N + (q & (s->N - 1))];
        owner[(size_t)r * s->N + (q & (s->N - 1))] = kNoOwner;
        if (who == kNoOwner) continue;  // not a load request (e.g. an open)
        if (who <= -2) {
          // a session's heap is closed on the device: its slot and budget
          // return, and the client waits for admission again
          const int32_t cid = -(who + 2);
          Client& c = cl[cid];
          note_open(L, -1);  // counted closed before its budget can be reused
          {
            std::lock_guard<std::mutex> g(s->slots_mu);
            s->free_slots.push_back(c.heap);
            s->held -= (int64_t)s->slot_bytes;
          }
          c.heap = -1;
          c.busy = false;
          --busy;
          ++out.sessions;
          if (!c.waiting.empty()) ++out.admission_waits;
          pending.push_back(cid);
          continue;
        }
        const int32_t cid = who;
        Client& c = cl[cid];
        ++out.completed;
        if (c.arrival >= t_warm && c.arrival < t_end) {
          out.lat_us.push_back((float)((tc - c.arrival) * 1e6));
          const CplEntry& e = ce[q & (s->N - 1)];
          const double q_us = (double)(e.t_pick - e.t_seen) * L.us_per_tick;
          const double s_us = (double)(e.t_done - e.t_pick) * L.us_per_tick;
          const double dev_us = (double)(e.t_done - e.t_seen) * L.us_per_tick;
          out.host_us.push_back((float)((c.submitted - c.arrival) * 1e6));
          out.queue_us.push_back((float)q_us);
          out.service_us.push_back((float)s_us);
          out.transit_us.push_back((float)((tc - c.submitted) * 1e6 - dev_us));
          ++out.measured;
        }
        if (tc >= t_warm && tc < t_end) ++out.in_window;
        if (c.op == HDA_OP_ALLOC) {
          if (res >= 0) {
            ++out.alloc_ok;
            c.live.push_back({c.issued_at + c.life, res});
            std::push_heap(c.live.begin(), c.live.end(), cmp);
          } else if (res == HDA_FAIL) {
            ++out.alloc_fail;
          } else {
            ++out.errors;
          }
        } else {
          ++out.frees;
          if (res != HDA_OK) ++out.errors;
        }
        if (cid < cfg.log_clients && cfg.log && cfg.log_len) {
          const int64_t n = cfg.log_len[cid];
          if (n < cfg.log_cap) {
            int64_t* e = cfg.log + ((int64_t)cid * cfg.log_cap + n) * 3;
            e[0] = c.op; e[1] = c.arg; e[2] = res;
            cfg.log_len[cid] = n + 1;
          }
        }
        c.busy = false;
        --busy;
        if (cfg.session_len > 0 && c.session_left <= 0) {
          // the session ends: close its heap (completion handled above)
          const uint64_t t = push_load(s, c.heap, kSrvClose, 0, 0);
          if (t == hda_server::kFullRing) {
            ++out.errors;
          } else {
            owner[(t >> 40) * s->N + (t & (s->N - 1))] = close_mark(cid);
            c.busy = true;
            ++busy;
          }
        } else if (!c.waiting.empty()) {
          const double a = c.waiting.front();
          c.waiting.pop_front();
          if (issue(L, c, cid, a, owner)) {
            ++busy;
            ++out.issued;
          } else {
            c.busy = false;
            ++out.errors;
          }
        }
      }
      // the ring's entries up to ct are consumed and free for reuse
      {
        std::lock_guard<std::mutex> g(s->rs[r].mu);
        for (uint64_t q = seen[k]; q < ct; ++q)
          s->rs[r].results[q & (s->N - 1)] = ce[q & (s->N - 1)].result;
        s->rs[r].harvested = ct;
      }
      seen[k] = ct;
      did = true;
    }
    if (now >= t_end && busy == 0) break;
    if (now >= t_end + 10.0) {  // completions stopped arriving: give up
      out.errors += busy;
      break;
    }
    if (!did) std::this_thread::yield();
  }
}

}  // namespace

extern "C" int hda_serve_load(hda_server* s, const hda_load_config* cfg, hda_load_report* rep) {
  if (!s || !cfg || !rep || cfg->clients <= 0 || cfg->rate <= 0 || cfg->measure_s <= 0 ||
      cfg->warmup_s < 0 || cfg->pow2_lo > cfg->pow2_hi || cfg->size_lo == 0 ||
      cfg->size_lo > cfg->size_hi || cfg->arena_lo == 0 || cfg->arena_lo > cfg->arena_hi ||
      cfg->lifetime_mean <= 0 || cfg->session_len < 0 ||
      (cfg->log_clients > 0 && (!cfg->log || !cfg->log_len)))
    return HDA_E_INVAL;
  std::memset(rep, 0, sizeof(*rep));
  int T = cfg->threads > 0 ? cfg->threads : 4;
  while (T > 1 && s->G % T) --T;
  std::vector<Client> clients(cfg->clients);
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device) != hipSuccess ||
      khz <= 0)
    khz = 100000;
  LoadShared L;
  L.cfg = cfg;
  L.s = s;
  L.clients = &clients;
  L.us_per_tick = 1e3 / (double)khz;
  for (int32_t c = 0; c < cfg->clients; ++c) {
    Client& k = clients[c];
    k.rng.x = cfg->seed * 0x2545f4914f6cdd1dull + (uint64_t)c * 0x9e3779b97f4a7c15ull;
    uint64_t a = log_uniform(k.rng, (double)cfg->arena_lo, (double)cfg->arena_hi);
    a = a / cfg->align * cfg->align;
    if (a == 0) a = cfg->align;
    k.arena = a;
    if (c < cfg->log_clients) cfg->log_len[c] = 0;
    if (cfg->session_len > 0) continue;  // sessions: admitted by the load threads
    const int rc = hda_serve_open(s, a, cfg->align, cfg->algo, &k.heap);
    if (rc != HDA_OK) {
      for (int32_t j = 0; j < c; ++j) hda_serve_close(s, clients[j].heap);
      return rc;
    }
    note_open(L, 1);
    if (c < cfg->log_clients) {  // row 0 of a client's log: (0, arena, align)
      int64_t* e = cfg->log + (int64_t)c * cfg->log_cap * 3;
      e[0] = 0; e[1] = (int64_t)a; e[2] = (int64_t)cfg->align;
      cfg->log_len[c] = cfg->log_cap > 0 ? 1 : 0;
    }
  }
  // the opens are queued ahead of every request on the same rings
  const double t0 = now_s();
  L.t_warm = t0 + cfg->warmup_s;
  L.t_end = t0 + cfg->warmup_s + cfg->measure_s;
  std::vector<ThreadOut> outs(T);
  std::vector<std::thread> th;
  for (int p = 0; p < T; ++p) th.emplace_back(run_thread, std::ref(L), p, T, std::ref(outs[p]));
  for (auto& t : th) t.join();
  std::vector<float> lat, hq, dq, ds, tr;
  for (auto& o : outs) {
    hq.insert(hq.end(), o.host_us.begin(), o.host_us.end());
    dq.insert(dq.end(), o.queue_us.begin(), o.queue_us.end());
    ds.insert(ds.end(), o.service_us.begin(), o.service_us.end());
    tr.insert(tr.end(), o.transit_us.begin(), o.transit_us.end());
    rep->issued += o.issued; rep->completed += o.completed; rep->measured += o.measured;
    rep->alloc_ok += o.alloc_ok; rep->alloc_fail += o.alloc_fail; rep->frees += o.frees;
    rep->errors += o.errors;
    rep->sessions += o.sessions;
    rep->admission_waits += o.admission_waits;
    rep->throughput += (double)o.in_window;
    lat.insert(lat.end(), o.lat_us.begin(), o.lat_us.end());
  }
  rep->max_open = L.open_max.load();
  rep->slot_bytes = (int64_t)s->slot_bytes;
  rep->window_s = cfg->measure_s;
  rep->throughput /= cfg->measure_s;
  auto pct = [](std::vector<float>& v, double f) {
    if (v.empty()) return 0.0;
    size_t k = (size_t)std::min<double>(v.size() - 1, std::floor(f * (v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return (double)v[k];
  };
  rep->host_p50_us = pct(hq, 0.5); rep->host_p99_us = pct(hq, 0.99);
  rep->queue_p50_us = pct(dq, 0.5); rep->queue_p99_us = pct(dq, 0.99);
  rep->service_p50_us = pct(ds, 0.5); rep->service_p99_us = pct(ds, 0.99);
  rep->transit_p50_us = pct(tr, 0.5); rep->transit_p99_us = pct(tr, 0.99);
  if (!lat.empty()) {
    auto q = [&](double f) { return pct(lat, f); };
    double sum = 0;
    for (float v : lat) sum += v;
    rep->mean_us = sum / lat.size();
    rep->p50_us = q(0.50);
    rep->p90_us = q(0.90);
    rep->p99_us = q(0.99);
    rep->p999_us = q(0.999);
    rep->max_us = *std::max_element(lat.begin(), lat.end());
  }
  if (cfg->close_heaps)
    for (auto& k : clients)
      if (k.heap >= 0) hda_serve_close(s, k.heap);
  return HDA_OK;
}

// Bytes of device metadata one admitted heap holds under `cfg` (what the
// metadata budget is counted in).
extern "C" int64_t hda_serve_slot_bytes(const hda_serve_config* cfg) {
  if (!cfg || cfg->slot_free < 0 || cfg->slot_live < 0) return HDA_E_INVAL;
  const uint32_t cf = (uint32_t)(((cfg->slot_free ? cfg->slot_free : 512) + 63) / 64 * 64);
  const uint32_t cl = (uint32_t)(((cfg->slot_live ? cfg->slot_live : 512) + 63) / 64 * 64);
  return (int64_t)((heap_bytes(cf, cl) + 255) / 256 * 256);
}
