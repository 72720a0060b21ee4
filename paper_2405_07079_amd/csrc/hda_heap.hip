// Single device-resident heaps driven call by call: heap_create / alloc /
// free / state.  The heap's registers and tables live in device memory; each
// call is one single-wave launch that loads the registers, runs one operation
// of the same core as the batched replay, and stores them back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "hda.h"
#include "hda_wave.h"
#include "hda_core.h"
#include "hda_heap_dev.h"
#include "hda_mem.h"

using namespace hda;

namespace {

enum : int { kOpInit = 0, kOpAlloc = 1, kOpFree = 2, kOpDump = 3, kOpFreePartial = 4 };

template <int ALGO>
__device__ void heap_call_t(HeapHdr* hd, int op, int64_t arg, int64_t* out, int64_t cap) {
  const Cold c = heap_cold(hd);
  WaveHeap<ALGO, 0, 0> w(c, load_regs(hd), hd->cf, hd->cl);
  int64_t r = 0;
  if (op == kOpInit) {
    w.init();
  } else if (op == kOpAlloc) {
    r = arg < 0 ? kEInval : w.alloc_bytes(arg);
  } else if (op == kOpFree) {
    r = w.free_offset(arg);
  } else if (op == kOpFreePartial) {
    r = w.free_partial(arg);
  } else {
    r = w.dump(out + 1, cap - 1);
  }
  store_regs(hd, w.h);
  if (lane_id() == 0) out[0] = r;
}

__global__ void heap_call(HeapHdr* hd, int op, int64_t arg, int64_t* out, int64_t cap) {
  switch (hd->algo) {
    case kFirstFit: heap_call_t<kFirstFit>(hd, op, arg, out, cap); break;
    case kNextFit: heap_call_t<kNextFit>(hd, op, arg, out, cap); break;
    case kBestFit: heap_call_t<kBestFit>(hd, op, arg, out, cap); break;
    case kSegFit: heap_call_t<kSegFit>(hd, op, arg, out, cap); break;
    default: heap_call_t<kTlsf>(hd, op, arg, out, cap); break;
  }
}

std::atomic<int64_t> g_budget{0};  // 0 = unlimited
std::atomic<int64_t> g_held{0};

// The installed device allocator (none: hipMalloc / hipFree) and the number
// of buffers obtained from it that are still held.
struct Allocator {
  std::mutex mu;
  hda_dev_alloc_fn alloc = nullptr;
  hda_dev_free_fn release = nullptr;
  void* ctx = nullptr;
  int64_t held = 0;
};
Allocator& allocator() {
  static Allocator a;
  return a;
}

}  // namespace

namespace hda {

void* dev_alloc(size_t bytes) {
  Allocator& a = allocator();
  std::lock_guard<std::mutex> g(a.mu);
  void* p = nullptr;
  if (a.alloc) {
    p = a.alloc(bytes, a.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) ++a.held;
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  Allocator& a = allocator();
  std::lock_guard<std::mutex> g(a.mu);
  if (a.release) a.release(p, a.ctx);
  else (void)hipFree(p);
  --a.held;
}

hipStream_t lib_stream() {
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

}  // namespace hda

struct hda_heap {
  HeapHdr* dev = nullptr;      // header + tables (device)
  int64_t* io = nullptr;       // device result / dump buffer
  size_t io_words = 0;
  size_t bytes = 0;            // metadata bytes charged to the budget
  hipStream_t stream = nullptr;  // the library's stream of the heap's device
  int algo = 0;
  uint64_t arena = 0, align = 0;
  uint32_t cap = 0;            // table capacities (entries)
  std::mutex mu;
};

namespace {

int call(hda_heap* h, int op, int64_t arg, int64_t* result, int64_t* dump, size_t cap,
         size_t* len) {
  std::lock_guard<std::mutex> g(h->mu);
  const size_t need_io = (op == kOpDump) ? cap + 1 : 1;
  if (need_io > h->io_words) {
    if (h->io) {
      (void)hipStreamSynchronize(h->stream);
      dev_free(h->io);
    }
    h->io = nullptr;
    h->io_words = 0;
    h->io = static_cast<int64_t*>(dev_alloc(need_io * 8));
    if (!h->io) return HDA_E_DEVICE;
    h->io_words = need_io;
  }
  hipLaunchKernelGGL(heap_call, dim3(1), dim3(64), 0, h->stream, h->dev, op, arg, h->io,
                     (int64_t)need_io);
  if (hipGetLastError() != hipSuccess) return HDA_E_DEVICE;
  int64_t r = 0;
  if (hipMemcpyAsync(&r, h->io, 8, hipMemcpyDeviceToHost, h->stream) != hipSuccess)
    return HDA_E_DEVICE;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return HDA_E_DEVICE;
  if (op == kOpDump) {
    *len = (size_t)r;
    if ((size_t)r > cap) return HDA_E_RANGE;
    if (r > 0 && (hipMemcpyAsync(dump, h->io + 1, (size_t)r * 8, hipMemcpyDeviceToHost,
                                 h->stream) != hipSuccess ||
                  hipStreamSynchronize(h->stream) != hipSuccess))
      return HDA_E_DEVICE;
    return HDA_OK;
  }
  *result = r;
  return HDA_OK;
}

}  // namespace


namespace {

int floor_log2_u64(uint64_t x) { return 63 - __builtin_clzll(x); }

// TLSF list of a block of b bytes (fl * 32 + sl, as in the state format).
uint32_t tlsf_list(uint64_t b) {
  const int fl = floor_log2_u64(b);
  const uint64_t sl = fl >= (int)kSli ? (b >> (fl - (int)kSli)) - kNsl : (b << ((int)kSli - fl)) - kNsl;
  return (uint32_t)fl * kNsl + (uint32_t)sl;
}

// Check a canonical state (format in hda.h) for heap h and lay it out as the
// device image of that heap: header, free table with push stamps, live
// table.  The class lists' head-to-tail order becomes descending stamps
// within each class, which is how the device core orders a list.  Returns
// HDA_OK, HDA_E_INVAL (malformed, or not a state of this heap's arena,
// alignment and algorithm) or HDA_E_NOMETA (more blocks than the tables
// hold).
int build_image(const hda_heap* h, const int64_t* buf, size_t len, std::vector<uint8_t>& img) {
  const int64_t A = (int64_t)h->arena, g = (int64_t)h->align;
  const int algo = h->algo;
  const uint32_t shift = (uint32_t)__builtin_ctzll(h->align);
  size_t p = 0;
  auto word = [&](int64_t& v) {
    if (p >= len) return false;
    v = buf[p++];
    return true;
  };
  struct Blk { int64_t a, s; bool free; };
  std::vector<Blk> all;
  int64_t nf = 0, nl = 0;
  if (!word(nf) || nf < 0 || (uint64_t)nf > (len - p) / 2) return HDA_E_INVAL;
  std::vector<Blk> fr((size_t)nf);
  for (int64_t i = 0; i < nf; ++i) {
    word(fr[i].a);
    word(fr[i].s);
    fr[i].free = true;
    if (i > 0 && fr[i].a <= fr[i - 1].a) return HDA_E_INVAL;  // address order
  }
  if (!word(nl) || nl < 0 || (uint64_t)nl > (len - p) / 2) return HDA_E_INVAL;
  std::vector<Blk> lv((size_t)nl);
  for (int64_t i = 0; i < nl; ++i) {
    word(lv[i].a);
    word(lv[i].s);
    lv[i].free = false;
  }
  int64_t rover = 0, bitmap = 0;
  if (!word(rover) || !word(bitmap)) return HDA_E_INVAL;
  // tiling of [0, A): aligned, positive, contiguous, no two free blocks adjacent
  all = fr;
  all.insert(all.end(), lv.begin(), lv.end());
  std::sort(all.begin(), all.end(), [](const Blk& x, const Blk& y) { return x.a < y.a; });
  int64_t pos = 0;
  for (size_t i = 0; i < all.size(); ++i) {
    const Blk& b = all[i];
    if (b.a != pos || b.s <= 0 || b.s % g || b.s > A - pos) return HDA_E_INVAL;
    if (i > 0 && b.free && all[i - 1].free) return HDA_E_INVAL;
    pos += b.s;
  }
  if (pos != A) return HDA_E_INVAL;
  if (algo == HDA_NEXT_FIT) {
    if (rover < 0 || rover > A || rover % g) return HDA_E_INVAL;
  } else if (rover != -1) {
    return HDA_E_INVAL;
  }
  // class lists (segregated fit: 64 classes of floor(log2 bytes); TLSF: 2,048)
  const bool seg = algo == HDA_SEG_FIT || algo == HDA_TLSF;
  const uint32_t n_lists = algo == HDA_SEG_FIT ? 64u : algo == HDA_TLSF ? kTlsfClasses : 0u;
  std::vector<uint32_t> stamp((size_t)nf, 0u);
  uint64_t want_bitmap = 0;
  uint32_t clock = 1;
  for (uint32_t c = 0; c < n_lists; ++c) {
    int64_t n = 0;
    if (!word(n) || n < 0 || (uint64_t)n > len - p) return HDA_E_INVAL;
    for (int64_t k = 0; k < n; ++k) {
      int64_t a = 0;
      word(a);
      const auto it = std::lower_bound(fr.begin(), fr.end(), a,
                                       [](const Blk& b, int64_t x) { return b.a < x; });
      if (it == fr.end() || it->a != a) return HDA_E_INVAL;  // not a free block
      const size_t i = (size_t)(it - fr.begin());
      const uint64_t b = (uint64_t)it->s;
      const uint32_t cls = algo == HDA_SEG_FIT ? (uint32_t)floor_log2_u64(b) : tlsf_list(b);
      if (cls != c || stamp[i] != 0u) return HDA_E_INVAL;  // wrong list or listed twice
      stamp[i] = clock + (uint32_t)(n - 1 - k);            // head: the newest push
    }
    clock += (uint32_t)n;
    if (n > 0) want_bitmap |= 1ull << (algo == HDA_SEG_FIT ? c : c / kNsl);
  }
  if (p != len) return HDA_E_INVAL;
  if (seg) {
    if ((uint64_t)bitmap != want_bitmap) return HDA_E_INVAL;
    for (uint32_t st : stamp)
      if (st == 0u) return HDA_E_INVAL;  // a free block in no list
  } else if (bitmap != 0) {
    return HDA_E_INVAL;
  }
  if ((uint64_t)nf > h->cap || (uint64_t)nl > h->cap) return HDA_E_NOMETA;
  // the device image
  img.assign(heap_bytes(h->cap, h->cap), 0);
  HeapHdr hdr;
  std::memset(&hdr, 0, sizeof(hdr));
  hdr.F = (uint32_t)nf;
  hdr.L = (uint32_t)nl;
  hdr.ag = (uint32_t)((uint64_t)A >> shift);
  hdr.shift = shift;
  hdr.rover = algo == HDA_NEXT_FIT ? (uint32_t)((uint64_t)rover >> shift) : 0u;
  hdr.clock = clock;
  hdr.algo = algo;
  hdr.arena = A;
  hdr.cf = h->cap;
  hdr.cl = h->cap;
  Ent* fe = reinterpret_cast<Ent*>(img.data() + sizeof(HeapHdr));
  uint32_t* fst = reinterpret_cast<uint32_t*>(img.data() + sizeof(HeapHdr) + (size_t)h->cap * 8);
  Ent* le = reinterpret_cast<Ent*>(img.data() + sizeof(HeapHdr) + (size_t)h->cap * 12);
  for (int64_t i = 0; i < nf; ++i) {
    const uint32_t a = (uint32_t)((uint64_t)fr[i].a >> shift), sg = (uint32_t)((uint64_t)fr[i].s >> shift);
    fe[i] = ((uint64_t)sg << 32) | a;
    fst[i] = stamp[i];
    if (algo == HDA_SEG_FIT) hdr.cnt[floor_log2_u64((uint64_t)fr[i].s)]++;
  }
  for (int64_t i = 0; i < nl; ++i)
    le[i] = ((uint64_t)((uint64_t)lv[i].s >> shift) << 32) | (uint32_t)((uint64_t)lv[i].a >> shift);
  std::memcpy(img.data(), &hdr, sizeof(hdr));
  return HDA_OK;
}

}  // namespace

extern "C" {

int hda_heap_create(uint64_t arena_bytes, uint64_t align, int algo, uint32_t meta_cap,
                    hda_heap** out) {
  if (!out) return HDA_E_INVAL;
  *out = nullptr;
  if (algo < HDA_FIRST_FIT || algo > HDA_TLSF) return HDA_E_INVAL;
  if (align == 0 || (align & (align - 1)) || arena_bytes == 0 || arena_bytes % align ||
      arena_bytes > (uint64_t)INT64_MAX || arena_bytes / align >= (uint64_t(1) << 32))
    return HDA_E_INVAL;
  const uint32_t cap = ((meta_cap ? meta_cap : 4096u) + 63u) / 64u * 64u;
  const size_t bytes = heap_bytes(cap, cap);
  const int64_t budget = g_budget.load();
  const int64_t held = g_held.fetch_add((int64_t)bytes) + (int64_t)bytes;
  if (budget > 0 && held > budget) {
    g_held.fetch_sub((int64_t)bytes);
    return HDA_E_NOMETA;
  }
  hda_heap* h = new (std::nothrow) hda_heap;
  if (!h) { g_held.fetch_sub((int64_t)bytes); return HDA_E_DEVICE; }
  h->bytes = bytes;
  h->algo = algo;
  h->arena = arena_bytes;
  h->align = align;
  h->cap = cap;
  h->stream = lib_stream();
  h->dev = h->stream ? static_cast<HeapHdr*>(dev_alloc(bytes)) : nullptr;
  if (!h->dev) {
    g_held.fetch_sub((int64_t)bytes);
    delete h;
    return HDA_E_DEVICE;
  }
  HeapHdr hdr;
  std::memset(&hdr, 0, sizeof(hdr));
  hdr.algo = algo;
  hdr.arena = (int64_t)arena_bytes;
  hdr.shift = (uint32_t)__builtin_ctzll(align);
  hdr.ag = (uint32_t)(arena_bytes >> hdr.shift);
  hdr.cf = cap;
  hdr.cl = cap;
  int64_t dummy = 0;
  if (hipMemcpyAsync(h->dev, &hdr, sizeof(hdr), hipMemcpyHostToDevice, h->stream) !=
          hipSuccess ||
      call(h, kOpInit, 0, &dummy, nullptr, 0, nullptr) != HDA_OK) {
    hda_heap_destroy(h);
    return HDA_E_DEVICE;
  }
  *out = h;
  return HDA_OK;
}

int hda_heap_destroy(hda_heap* h) {
  if (!h) return HDA_E_INVAL;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  dev_free(h->dev);
  dev_free(h->io);
  g_held.fetch_sub((int64_t)h->bytes);
  delete h;
  return HDA_OK;
}

int64_t hda_alloc(hda_heap* h, uint64_t size) {
  if (!h || size > (uint64_t)INT64_MAX) return HDA_E_INVAL;
  int64_t r = 0;
  const int rc = call(h, kOpAlloc, (int64_t)size, &r, nullptr, 0, nullptr);
  return rc != HDA_OK ? rc : r;
}

int hda_free(hda_heap* h, int64_t offset) {
  if (!h) return HDA_E_INVAL;
  int64_t r = 0;
  const int rc = call(h, kOpFree, offset, &r, nullptr, 0, nullptr);
  return rc != HDA_OK ? rc : (int)r;
}

int hda_free_partial(hda_heap* h, int64_t offset) {
  if (!h) return HDA_E_INVAL;
  int64_t r = 0;
  const int rc = call(h, kOpFreePartial, offset, &r, nullptr, 0, nullptr);
  return rc != HDA_OK ? rc : (int)r;
}

int hda_heap_load(hda_heap* h, const int64_t* buf, size_t len) {
  if (!h || (len && !buf)) return HDA_E_INVAL;
  std::vector<uint8_t> img;
  const int rc = build_image(h, buf, len, img);
  if (rc != HDA_OK) return rc;
  std::lock_guard<std::mutex> g(h->mu);
  if (hipMemcpyAsync(h->dev, img.data(), img.size(), hipMemcpyHostToDevice, h->stream) !=
          hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return HDA_E_DEVICE;
  return HDA_OK;
}

int hda_set_device_allocator(hda_dev_alloc_fn alloc, hda_dev_free_fn release, void* ctx) {
  if ((alloc == nullptr) != (release == nullptr)) return HDA_E_INVAL;
  Allocator& a = allocator();
  std::lock_guard<std::mutex> g(a.mu);
  if (a.held != 0) return HDA_E_BUSY;  // buffers of the current allocator are still held
  a.alloc = alloc;
  a.release = release;
  a.ctx = ctx;
  return HDA_OK;
}

int hda_heap_state(const hda_heap* h, int64_t* buf, size_t cap, size_t* len) {
  if (!h || !len || (cap && !buf)) return HDA_E_INVAL;
  return call(const_cast<hda_heap*>(h), kOpDump, 0, nullptr, buf, cap, len);
}

int64_t hda_set_meta_budget(int64_t bytes) {
  g_budget.store(bytes > 0 ? bytes : 0);
  return g_held.load();
}

const char* hda_strerror(int code) {
  switch (code) {
    case HDA_OK: return "ok";
    case HDA_FAIL: return "allocation failed: no free block fits";
    case HDA_E_INVAL: return "invalid argument";
    case HDA_E_BADFREE:
      return "free of an offset that is not a live block's start (partial free: in no live block)";
    case HDA_E_NOMETA: return "metadata capacity or budget exhausted";
    case HDA_E_DEVICE: return "HIP runtime error";
    case HDA_E_BUSY: return "resource busy";
    case HDA_E_RANGE: return "output buffer too small";
    default: return "unknown error";
  }
}

}  // extern "C"
