// Device memory and streams the library uses for itself (host side).
//
// Every device buffer the library keeps -- call-by-call heap metadata and
// result buffers, the service's heap pool, the autotuner's trial batch --
// comes from dev_alloc / dev_free, which call the allocator installed with
// hda_set_device_allocator (for instance the caller's caching allocator), or
// hipMalloc / hipFree when none is installed.  Call-by-call heaps share one
// stream per device, created on first use.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace hda {

void* dev_alloc(size_t bytes);
void dev_free(void* p);
// The library's stream on the current device (nullptr on failure).
hipStream_t lib_stream();

}  // namespace hda
