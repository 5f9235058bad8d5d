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

// Float partner value of lane ^ m (m < 64).
__device__ __forceinline__ float xor_f(float v, int m, int lane) { return bperm_f(v, lane ^ m); }

__device__ __forceinline__ uint64_t xor64(uint64_t v, int m, int lane) {
  return bperm64(v, lane ^ m);
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
