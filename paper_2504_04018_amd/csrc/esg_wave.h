// Wave64 primitives for gfx950: lane ids, cross-lane moves, ordered keys.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace esgk {

constexpr int kWave = 64;
constexpr uint64_t kKeyInf = ~0ull;
constexpr uint32_t kNoNode = 0xFFFFFFFFu;

__device__ __forceinline__ int lane_id() {
  return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ int rank_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t bperm(uint32_t v, int src_lane) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)v);
}

__device__ __forceinline__ float bperm_f(float v, int src_lane) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}

__device__ __forceinline__ uint64_t bperm64(uint64_t v, int src_lane) {
  uint32_t lo = bperm((uint32_t)v, src_lane);
  uint32_t hi = bperm((uint32_t)(v >> 32), src_lane);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
  uint32_t lo = readlane((uint32_t)v, lane);
  uint32_t hi = readlane((uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t first_lane(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Orders LDS traffic of one wave: every lane's earlier LDS writes are
// visible to every lane's later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value held by lane ^ m (m a power of two below 64, a compile-time
// constant after unrolling).  Xor 1 and 2 are DPP quad permutes, 4 and 8
// DPP row shifts (lanes with the bit clear read lane+m, the others
// lane-m), 16 a ds_swizzle inside each half wave, 32 a permlane32 swap.
__device__ __forceinline__ uint32_t xor_u32(uint32_t v, int m, int lane) {
  switch (m) {
    case 1:
      return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
    case 2:
      return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
    case 4: {
      uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x104, 0xF, 0xF, false);
      uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x114, 0xF, 0xF, false);
      return (lane & 4) ? dn : up;
    }
    case 8: {
      uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x108, 0xF, 0xF, false);
      uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x118, 0xF, 0xF, false);
      return (lane & 8) ? dn : up;
    }
    case 16:
      return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);
    default: {
      auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
      return lane < 32 ? p[1] : p[0];
    }
  }
}

__device__ __forceinline__ float xor_f(float v, int m, int lane) {
  return __uint_as_float(xor_u32(__float_as_uint(v), m, lane));
}

__device__ __forceinline__ uint64_t xor64(uint64_t v, int m, int lane) {
  uint32_t lo = xor_u32((uint32_t)v, m, lane);
  uint32_t hi = xor_u32((uint32_t)(v >> 32), m, lane);
  return ((uint64_t)hi << 32) | lo;
}

// Value held by lane + 1 (lane 63 receives garbage: callers overwrite it).
__device__ __forceinline__ uint64_t next_lane64(uint64_t v) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, 0x130, 0xF, 0xF, false);
  uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), 0x130, 0xF, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}

// Value held by lane - 1 (lane 0 receives garbage: callers overwrite it).
__device__ __forceinline__ uint64_t prev_lane64(uint64_t v) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, 0x138, 0xF, 0xF, false);
  uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), 0x138, 0xF, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t kmin(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t kmax(uint64_t a, uint64_t b) { return a < b ? b : a; }

// A candidate key: non-negative float distance bits above the position, so
// unsigned comparison of keys is the (distance, position) order.
__device__ __forceinline__ uint64_t make_key(float dist, uint32_t pos) {
  return ((uint64_t)__float_as_uint(dist) << 32) | pos;
}
__device__ __forceinline__ uint32_t key_pos(uint64_t k) { return (uint32_t)k; }
__device__ __forceinline__ float key_dist(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }

}  // namespace esgk
