// Single device-resident heaps driven call by call: heap_create / alloc /
// free / state.  The heap's registers and tables live in device memory; each
// call is one single-wave launch that loads the registers, runs one operation
// of the same core as the batched replay, and stores them back.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>

#include "hda.h"
#include "hda_wave.h"
#include "hda_core.h"
#include "hda_heap_dev.h"

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

}  // namespace

struct hda_heap {
  HeapHdr* dev = nullptr;      // header + tables (device)
  int64_t* io = nullptr;       // device result / dump buffer
  size_t io_words = 0;
  size_t bytes = 0;            // metadata bytes charged to the budget
  hipStream_t stream = nullptr;
  std::mutex mu;
};

namespace {

int call(hda_heap* h, int op, int64_t arg, int64_t* result, int64_t* dump, size_t cap,
         size_t* len) {
  std::lock_guard<std::mutex> g(h->mu);
  const size_t need_io = (op == kOpDump) ? cap + 1 : 1;
  if (need_io > h->io_words) {
    if (h->io) (void)hipFree(h->io);
    h->io = nullptr;
    h->io_words = 0;
    if (hipMalloc(&h->io, need_io * 8) != hipSuccess) return HDA_E_DEVICE;
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
    if (r > 0 && hipMemcpy(dump, h->io + 1, (size_t)r * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return HDA_E_DEVICE;
    return HDA_OK;
  }
  *result = r;
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
  if (hipMalloc(&h->dev, bytes) != hipSuccess ||
      hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
    if (h->dev) (void)hipFree(h->dev);
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
  if (hipMemcpy(h->dev, &hdr, sizeof(hdr), hipMemcpyHostToDevice) != hipSuccess ||
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
  if (h->dev) (void)hipFree(h->dev);
  if (h->io) (void)hipFree(h->io);
  if (h->stream) (void)hipStreamDestroy(h->stream);
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
