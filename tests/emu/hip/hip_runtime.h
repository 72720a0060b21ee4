// Host stand-in for the few HIP names the device core uses, so that the core
// can be compiled by g++ and run under the lockstep wave emulation.
#pragma once
#include <algorithm>
#include <cstddef>
#include <cstdint>

#define __device__
#define __host__
#define __forceinline__ inline

struct uint2 {
  uint32_t x, y;
};
inline uint2 make_uint2(uint32_t x, uint32_t y) { return uint2{x, y}; }
using std::max;
using std::min;

// one heap runs at a time on one host thread: a plain read-modify-write
inline uint32_t atomicAdd(uint32_t* p, uint32_t v) {
  const uint32_t o = *p;
  *p = o + v;
  return o;
}
