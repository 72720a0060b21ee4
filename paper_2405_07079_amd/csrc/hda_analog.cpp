// Per-call latency harness for the paper's comparison with the vendor's
// allocation calls (Sec. VI), rebuilt for this device: one request stream
// replayed call by call (a) through hipMalloc / hipFree and (b) through one
// of this library's heaps (hda_alloc / hda_free, one launch per call).  Both
// sides free the same victims: a free request carries a 32-bit draw r and
// frees live[(r * L) >> 32] of the live blocks in allocation order, the last
// one moving into the hole.  Used by the benchmark only; not part of the
// library's interface.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <vector>

#include "hda.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// after(i) runs after request i, outside the timed region
template <typename Alloc, typename Free, typename After>
int replay(const int64_t* req, int64_t n, int64_t* lat_ns, int64_t* res, Alloc alloc,
           Free release, After after) {
  std::vector<int64_t> live;  // handles in allocation order
  for (int64_t i = 0; i < n; ++i) {
    const int64_t q = req[i];
    if (q >= 0) {
      const int64_t t0 = now_ns();
      const int64_t h = alloc(q);
      lat_ns[i] = now_ns() - t0;
      res[i] = h;
      if (h >= 0) live.push_back(h);
    } else if (live.empty()) {
      lat_ns[i] = 0;
      res[i] = -1;
    } else {
      const uint64_t r = (uint32_t)~(uint64_t)q;
      const size_t k = (size_t)((r * live.size()) >> 32);
      const int64_t h = live[k];
      const int64_t t0 = now_ns();
      const int rc = release(h);
      lat_ns[i] = now_ns() - t0;
      if (rc != 0) return rc;
      res[i] = h;
      live[k] = live.back();
      live.pop_back();
    }
    after(i);
  }
  return 0;
}

}  // namespace

extern "C" {

// hipMalloc / hipFree.  res receives 0 for a successful request (a pointer
// is not an offset), -1 for a failed allocation or a free with nothing live.  used_bytes, if not null,
// receives the device memory in use after each request (hipMemGetInfo; this
// slows the replay, so latencies come from a run without it).  Everything
// still allocated at the end is freed.  Returns 0 or a HIP error code.
int hda_analog_vendor(const int64_t* req, int64_t n, int64_t* lat_ns, int64_t* res,
                      int64_t* used_bytes) {
  std::vector<void*> ptrs;
  const int rc = replay(
      req, n, lat_ns, res,
      [&](int64_t q) -> int64_t {
        void* p = nullptr;
        if (hipMalloc(&p, (size_t)(q > 0 ? q : 1)) != hipSuccess) {
          (void)hipGetLastError();
          return -1;
        }
        ptrs.push_back(p);
        return (int64_t)(ptrs.size() - 1);
      },
      [&](int64_t h) -> int {
        const hipError_t e = hipFree(ptrs[(size_t)h]);
        ptrs[(size_t)h] = nullptr;
        return e == hipSuccess ? 0 : (int)e;
      },
      [&](int64_t i) {
        if (!used_bytes) return;
        size_t fr = 0, tot = 0;
        used_bytes[i] = hipMemGetInfo(&fr, &tot) == hipSuccess ? (int64_t)(tot - fr) : -1;
      });
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int64_t i = 0; i < n; ++i) res[i] = res[i] >= 0 ? 0 : -1;
  return rc;
}

// One heap of `arena` bytes (algorithm `algo`, alignment `align`, table
// capacity `meta_cap`) driven call by call.  res receives each request's
// result (byte offset or -1 for an allocation, the freed offset for a free).
int hda_analog_heap(const int64_t* req, int64_t n, uint64_t arena, uint64_t align, int algo,
                    uint32_t meta_cap, int64_t* lat_ns, int64_t* res) {
  hda_heap* h = nullptr;
  int rc = hda_heap_create(arena, align, algo, meta_cap, &h);
  if (rc != HDA_OK) return rc;
  rc = replay(
      req, n, lat_ns, res, [&](int64_t q) -> int64_t { return hda_alloc(h, (uint64_t)q); },
      [&](int64_t off) -> int { return hda_free(h, off); }, [](int64_t) {});
  hda_heap_destroy(h);
  return rc;
}

}  // extern "C"
