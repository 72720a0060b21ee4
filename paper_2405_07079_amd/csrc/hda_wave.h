// Wavefront primitives for gfx950 (64 lanes): lane id, ballot, readlane,
// readfirstlane, DPP row and wave shifts and ds_bpermute.  hda_core.h is written only
// against these names, so the same core can be compiled elsewhere with
// another definition of them (the test-suite runs it on the CPU with a
// lockstep emulation of a wave).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Pointers into LDS keep their address space, so accesses through them are
// ds_* instructions rather than generic (FLAT) ones.
#define HDA_LDS __attribute__((address_space(3)))
#define HDA_GLOBAL __attribute__((address_space(1)))

namespace hda {

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint64_t ballot(bool p) {
  return __builtin_amdgcn_ballot_w64(p);
}

__device__ __forceinline__ uint32_t rdlane(uint32_t v, uint32_t l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}

// Lane l of v receives the wave-uniform value x; other lanes keep v (one
// v_writelane; l is taken mod 64).
__device__ int hda_writelane(int x, int l, int v) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ uint32_t put_lane(uint32_t v, uint32_t l, uint32_t x) {
  return (uint32_t)hda_writelane((int)x, (int)l, (int)v);
}

// A value the optimiser may not trace back to the memory it was loaded
// from.  Selecting between table registers through it keeps a select chain
// from being folded into one load at a computed offset, which would pin the
// whole table in private (scratch) memory.
__device__ __forceinline__ uint32_t opaque(uint32_t v) {
  asm("" : "+v"(v));
  return v;
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Lane i of each 16-lane row receives src from lane i-K of the same row;
// lanes with no such source receive `old`.
template <int K>
__device__ __forceinline__ uint32_t row_shr(uint32_t old, uint32_t src) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x110 + K, 0xf, 0xf, false);
}

// Rows 1 and 3 receive lane 15 of the row below (lanes 15 and 47); rows 0
// and 2 keep `old` (DPP row_bcast:15 under row mask 0b1010).
__device__ __forceinline__ uint32_t row_bcast15(uint32_t old, uint32_t src) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x142, 0xa, 0xf, false);
}

// Rows 2 and 3 receive lane 31; rows 0 and 1 keep `old` (DPP row_bcast:31
// under row mask 0b1100).
__device__ __forceinline__ uint32_t row_bcast31(uint32_t old, uint32_t src) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x143, 0xc, 0xf, false);
}

// Whole-wave shifts by one lane (DPP wave_shr:1 / wave_shl:1): lane i
// receives src from lane i - 1 (shr1) or i + 1 (shl1); the lane with no
// source (0, resp. 63) receives `old`.
__device__ __forceinline__ uint32_t wave_shr1(uint32_t old, uint32_t src) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t wave_shl1(uint32_t old, uint32_t src) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x130, 0xf, 0xf, false);
}

__device__ __forceinline__ uint32_t shfl(uint32_t v, uint32_t src_lane) {
  return (uint32_t)__shfl((int)v, (int)src_lane);
}

// A value loaded from device memory is waited for here.  A table access
// that goes to LDS or to device memory by a uniform branch waits inside its
// device-memory branch, so that where the two paths join no device-memory
// load is outstanding, and the LDS path waits only for LDS -- not for the
// request prefetch or the result stores also counted by the same counter.
__device__ __forceinline__ void settle(uint32_t v) { asm volatile("" ::"v"(v)); }

// Ordering point between table accesses; lanes of a wave already execute in
// lockstep on the hardware, so there is nothing to do here.
__device__ __forceinline__ void wave_sync() {}

}  // namespace hda
