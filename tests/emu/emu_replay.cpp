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
  const Tables* t;
  int64_t heap;
  int done;
};
LaneJob g_job;

void lane_main() {
  replay_one_heap(*g_job.p, *g_job.t, g_job.heap);
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

}  // namespace

extern "C" int emu_replay(int64_t H, const int64_t* arena, const int64_t* align,
                          const int32_t* algo, const int64_t* req_off, const int64_t* req,
                          int64_t* res, int64_t* state, const int64_t* state_off,
                          int64_t* state_len, int32_t* status, uint32_t kf, uint32_t kl,
                          uint32_t cf, uint32_t cl, uint64_t* syncs) {
  ReplayParams p;
  std::memset(&p, 0, sizeof(p));
  p.arena = arena; p.align = align; p.algo = algo; p.req_off = req_off; p.req = req;
  p.res = res; p.state = state; p.state_off = state_off; p.state_len = state_len;
  p.status = status;
  p.kf = kf; p.kl = kl; p.cf = cf; p.cl = cl;
  std::vector<uint8_t> lds(size_t(kf) * 12 + size_t(kl) * 8 + 16);
  std::vector<Ent> gf(cf - kf + 64), gl(cl - kl + 64);
  std::vector<uint32_t> gst(cf - kf + 64);
  const size_t stack_bytes = 256 * 1024;
  std::vector<std::vector<uint8_t>> stacks(64, std::vector<uint8_t>(stack_bytes));
  EmuWave w;
  emu_wave = &w;
  for (int64_t h = 0; h < H; ++h) {
    // poison the tables so a read of an unwritten entry cannot look valid
    std::memset(lds.data(), 0xA5, lds.size());
    std::memset(gf.data(), 0xA5, gf.size() * sizeof(Ent));
    std::memset(gl.data(), 0xA5, gl.size() * sizeof(Ent));
    Tables t;
    t.lf = reinterpret_cast<Ent*>(lds.data());
    t.lst = reinterpret_cast<uint32_t*>(lds.data() + size_t(kf) * 8);
    t.ll = reinterpret_cast<Ent*>(lds.data() + size_t(kf) * 12);
    t.gf = gf.data(); t.gst = gst.data(); t.gl = gl.data();
    t.kf = kf; t.kl = kl; t.cf = cf; t.cl = cl;
    g_job = LaneJob{&p, &t, h, 0};
    w.syncs = 0;
    for (int l = 0; l < 64; ++l) {
      getcontext(&w.lane_ctx[l]);
      w.lane_ctx[l].uc_stack.ss_sp = stacks[l].data();
      w.lane_ctx[l].uc_stack.ss_size = stack_bytes;
      w.lane_ctx[l].uc_link = nullptr;
      makecontext(&w.lane_ctx[l], lane_main, 0);
    }
    emu_lane = 0;
    swapcontext(&w.main_ctx, &w.lane_ctx[0]);
    if (syncs) syncs[h] = w.syncs;
  }
  emu_wave = nullptr;
  return 0;
}
