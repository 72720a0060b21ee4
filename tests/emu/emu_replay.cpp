// CPU driver for the device replay core: runs one heap at a time as a wave of
// 64 lockstep fibers (see emu_wave.h), with "LDS" and spill tables in host
// memory.  Test infrastructure only.
#include <ucontext.h>

#include <cstdint>
#include <cstring>
#include <vector>

#include "emu_wave.h"
#include "hda_core.h"
#include "hda_replay_body.h"

namespace hda {
EmuWave* emu_wave = nullptr;
uint32_t emu_lane = 0;
}  // namespace hda

using namespace hda;

namespace {

struct LaneJob {
  const ReplayParams* p;
  const Cold* c;
  const LeanLds* lds;
  int64_t heap;
  int shape;
  int done;
  uint64_t* bits;        // bitmask allocator: flags, node summaries, live table
  uint64_t* nodes;
  Ent* live;
  uint64_t max_granules;
  uint8_t* ord_dev;      // ordered core: the wave's device slot
  uint64_t* lnodes;      // bitmask allocator: the "LDS" summaries (3) and live entries (40)
  Ent* llive;
};
LaneJob g_job;

template <int RF>
void lean_any(const ReplayParams& p, const LeanLds& lds, const Cold& c, int64_t heap) {
  switch (p.algo[heap]) {
    case kFirstFit: lean_one_heap<kFirstFit, RF>(p, lds, c, heap); break;
    case kNextFit: lean_one_heap<kNextFit, RF>(p, lds, c, heap); break;
    case kBestFit: lean_one_heap<kBestFit, RF>(p, lds, c, heap); break;
    case kSegFit: lean_one_heap<kSegFit, RF>(p, lds, c, heap); break;
    default: lean_one_heap<kTlsf, RF>(p, lds, c, heap); break;
  }
}

void lane_main() {
  switch (g_job.shape) {
    case 0: replay_any_heap<0, 0>(*g_job.p, *g_job.c, g_job.heap); break;
    case 1: replay_any_heap<1, 2>(*g_job.p, *g_job.c, g_job.heap); break;
    case 2: replay_any_heap<4, 8>(*g_job.p, *g_job.c, g_job.heap); break;
    case 3: lean_any<1>(*g_job.p, *g_job.lds, *g_job.c, g_job.heap); break;
    case 4: lean_any<4>(*g_job.p, *g_job.lds, *g_job.c, g_job.heap); break;
    case 6: ord_any_heap(*g_job.p, g_job.lds->base, g_job.ord_dev, g_job.heap); break;
    default:
      bitmap_one_heap(*g_job.p, g_job.bits, g_job.nodes, g_job.live, g_job.lnodes, 3u,
                      g_job.llive, 40u, g_job.max_granules,
                      g_job.heap);
      break;
  }
  // a finished lane keeps handing over until every lane has finished
  g_job.done++;
  for (;;) {
    const uint32_t me = emu_lane;
    if (g_job.done == 64) swapcontext(&emu_wave->lane_ctx[me], &emu_wave->main_ctx);
    const uint32_t next = (me + 1) & 63u;
    emu_lane = next;
    swapcontext(&emu_wave->lane_ctx[me], &emu_wave->lane_ctx[next]);
    emu_lane = me;
  }
}

const int kShapeRF[] = {0, 1, 4, 0, 0, 0, 0}, kShapeRL[] = {0, 2, 8, 0, 0, 0, 0};

// The bitmask allocator's node summaries recomputed granule by granule from
// the flags: bottom run | top run << 16 | longest run << 32 per 4,096
// granules.  True if every stored summary has the exact end runs and a
// longest run between the true one and 4,096 (allocations leave it as an
// upper bound).
bool summaries_valid(const uint64_t* bits, const uint64_t* nodes, uint64_t ag) {
  const uint64_t nw = (ag + 63u) / 64u, nn = (nw + 63u) / 64u;
  for (uint64_t n = 0; n < nn; ++n) {
    auto is_free = [&](uint64_t g) {  // g inside the node
      const uint64_t x = 4096u * n + g;
      return x < ag && ((bits[x / 64u] >> (x % 64u)) & 1u) != 0;
    };
    uint64_t bottom = 0, top = 0, best = 0, run = 0;
    while (bottom < 4096u && is_free(bottom)) ++bottom;
    while (top < 4096u && is_free(4095u - top)) ++top;
    for (uint64_t g = 0; g < 4096u; ++g) {
      run = is_free(g) ? run + 1u : 0u;
      best = run > best ? run : best;
    }
    if ((nodes[n] & 0xffffffffu) != (bottom | (top << 16))) return false;
    const uint64_t bound = nodes[n] >> 32;
    if (bound < best || bound > 4096u) return false;
  }
  return true;
}

// Run one heap as a wave of 64 fibers.
void run_wave(EmuWave& w, std::vector<std::vector<uint8_t>>& stacks) {
  w.syncs = 0;
  for (int l = 0; l < 64; ++l) {
    getcontext(&w.lane_ctx[l]);
    w.lane_ctx[l].uc_stack.ss_sp = stacks[l].data();
    w.lane_ctx[l].uc_stack.ss_size = stacks[l].size();
    w.lane_ctx[l].uc_link = nullptr;
    makecontext(&w.lane_ctx[l], lane_main, 0);
  }
  emu_lane = 0;
  swapcontext(&w.main_ctx, &w.lane_ctx[0]);
}

}  // namespace

// shape: general core with 0 = no register part, 1 = (1, 2) chunks, 2 = (4, 8)
// chunks in registers; lean core with 3 = one, 4 = four free chunks in
// registers, where a heap that outgrows its tiers moves to the general core
// on the same "LDS" plus spill tables (overflowed[h] = 1); 5 = the bitmask
// allocator (flags for the heap's own granules, cap_live live entries); 6 =
// the ordered core with a pool of 8 KiB + kf * 16 + kl * 8 bytes, kf * 16 of
// them meant for chunk slots.
// kf/kl: entries in "LDS"; cap_free/cap_live: capacities.
extern "C" int emu_replay(int64_t H, const int64_t* arena, const int64_t* align,
                          const int32_t* algo, const int64_t* req_off, const int64_t* req,
                          int64_t* res, int64_t* state, const int64_t* state_off,
                          int64_t* state_len, int32_t* status, int shape, uint32_t kf,
                          uint32_t kl, uint32_t cap_free, uint32_t cap_live, uint64_t* syncs,
                          uint8_t* overflowed) {
  ReplayParams p;
  std::memset(&p, 0, sizeof(p));
  p.arena = arena; p.align = align; p.algo = algo; p.req_off = req_off; p.req = req;
  p.res = res; p.state = state; p.state_off = state_off; p.state_len = state_len;
  p.status = status;
  const bool lean = shape == 3 || shape == 4;
  if (shape == 6) {
    // ordered core: its own pool and device slot, poisoned per heap
    p.cap_free = cap_free; p.cap_live = cap_live;
    p.ord_pool_bytes = 8192u + kf * 16u + kl * 8u;
    p.ord_slot_bytes = kf * 16u;
    std::vector<uint8_t> opool(size_t(p.ord_pool_bytes) + 16);
    std::vector<uint8_t> odev(size_t(ord_dev_bytes(cap_live)) + 16);
    const size_t stack_bytes = 256 * 1024;
    std::vector<std::vector<uint8_t>> stacks(64, std::vector<uint8_t>(stack_bytes));
    EmuWave w;
    emu_wave = &w;
    for (int64_t h = 0; h < H; ++h) {
      std::memset(opool.data(), 0xA5, opool.size());
      std::memset(odev.data(), 0xA5, odev.size());
      LeanLds ll;
      ll.base = opool.data();
      ll.bytes = p.ord_pool_bytes;
      g_job = LaneJob{&p, nullptr, &ll, h, shape, 0};
      g_job.ord_dev = odev.data();
      run_wave(w, stacks);
      if (syncs) syncs[h] = w.syncs;
    }
    emu_wave = nullptr;
    return 0;
  }
  // lean core: an LDS pool with room for kf 16-byte free and kl live entries;
  // the general core it may move to has no LDS part
  const uint32_t pool = kf * 16u + kl * 8u;
  if (lean) kf = kl = 0;
  const uint32_t hf = 64u * kShapeRF[shape], hl = 64u * kShapeRL[shape];
  const uint32_t coldF = cap_free > hf ? cap_free - hf : 0u;
  const uint32_t coldL = cap_live > hl ? cap_live - hl : 0u;
  kf = kf < coldF ? kf : coldF;
  kl = kl < coldL ? kl : coldL;
  p.cap_free = cap_free; p.cap_live = cap_live;
  p.kf = kf; p.kl = kl; p.sf = coldF - kf; p.sl = coldL - kl;
  std::vector<uint8_t> lds(size_t(kf) * 12 + size_t(kl) * 8 + 16);
  std::vector<uint8_t> pool_mem(size_t(pool) + 16);
  uint32_t migrated = 0;
  p.migrated = &migrated;
  std::vector<Ent> gf(p.sf + 64), gl(p.sl + 64);
  std::vector<uint32_t> gst(p.sf + 64);
  const size_t stack_bytes = 256 * 1024;
  std::vector<std::vector<uint8_t>> stacks(64, std::vector<uint8_t>(stack_bytes));
  EmuWave w;
  emu_wave = &w;
  for (int64_t h = 0; h < H; ++h) {
    // poison the tables so a read of an unwritten entry cannot look valid
    std::memset(lds.data(), 0xA5, lds.size());
    std::memset(gf.data(), 0xA5, gf.size() * sizeof(Ent));
    std::memset(gl.data(), 0xA5, gl.size() * sizeof(Ent));
    Cold c;
    c.lf = reinterpret_cast<Ent*>(lds.data());
    c.lst = reinterpret_cast<uint32_t*>(lds.data() + size_t(kf) * 8);
    c.ll = reinterpret_cast<Ent*>(lds.data() + size_t(kf) * 12);
    c.gf = gf.data(); c.gst = gst.data(); c.gl = gl.data();
    c.kf = kf; c.kl = kl; c.cf = coldF; c.cl = coldL;
    uint64_t n_sync = 0;
    if (lean) {
      std::memset(pool_mem.data(), 0xA5, pool_mem.size());
      LeanLds ll;
      ll.base = pool_mem.data();
      ll.bytes = pool;
      const uint32_t before = migrated;
      g_job = LaneJob{&p, &c, &ll, h, shape, 0};
      run_wave(w, stacks);
      n_sync = w.syncs;
      if (overflowed) overflowed[h] = migrated != before;
    } else if (shape == 5) {
      // poisoned flags and summaries past the heap's words and a poisoned
      // live table
      const uint64_t ag = (align[h] > 0 && arena[h] > 0) ? uint64_t(arena[h] / align[h]) : 1u;
      const uint64_t nw = (ag + 63u) / 64u;
      std::vector<uint64_t> bits(nw + 1u, 0xA5A5A5A5A5A5A5A5ull);
      std::vector<uint64_t> nodes((nw + 63u) / 64u + 1u, 0xA5A5A5A5A5A5A5A5ull);
      std::vector<Ent> live(size_t(cap_live) + 1u, 0xA5A5A5A5A5A5A5A5ull);
      // a few summaries and live entries in "LDS" (as the kernel keeps them),
      // so that both places are exercised
      std::vector<uint64_t> lnodes(3, 0xA5A5A5A5A5A5A5A5ull);
      std::vector<Ent> llive(40, 0xA5A5A5A5A5A5A5A5ull);
      g_job = LaneJob{&p, &c, nullptr, h, shape, 0, bits.data(), nodes.data(), live.data(), ag};
      g_job.lnodes = lnodes.data();
      g_job.llive = llive.data();
      run_wave(w, stacks);
      n_sync = w.syncs;
      for (uint64_t n = 0; n < 3 && n < nodes.size(); ++n) nodes[n] = lnodes[n];
      if (status[h] == 0 && !summaries_valid(bits.data(), nodes.data(), ag)) return 1;
    } else {
      g_job = LaneJob{&p, &c, nullptr, h, shape, 0};
      run_wave(w, stacks);
      n_sync = w.syncs;
    }
    if (syncs) syncs[h] = n_sync;
  }
  emu_wave = nullptr;
  return 0;
}
