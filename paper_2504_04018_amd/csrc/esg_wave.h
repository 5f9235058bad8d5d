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

// Forward permute: lane i's value lands in lane dst(i).  The destinations
// must form a permutation of the 64 lanes and every lane must be active,
// so that each lane is written exactly once.
__device__ __forceinline__ uint32_t push(uint32_t v, int dst) {
  return (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)v);
}

__device__ __forceinline__ uint64_t push64(uint64_t v, int dst) {
  const uint32_t lo = push((uint32_t)v, dst);
  const uint32_t hi = push((uint32_t)(v >> 32), dst);
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
// constant after unrolling).  Xor 1 and 2 are DPP quad permutes; xor 4 is a
// half-row mirror (lane ^ 7) followed by a quad reversal (^ 3), xor 8 a row
// mirror (^ 15) followed by a half-row mirror (^ 7): two DPP moves and no
// select; 16 is a ds_swizzle inside each half wave, 32 a permlane32 swap.
// Every DPP source lane is inside the row, so the bound-control form (which
// lets the compiler fold the move into the instruction that consumes it)
// returns the same values.
template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t xor_u32(uint32_t v, int m, int lane) {
  switch (m) {
    case 1:
      return (uint32_t)dpp<0xB1>((int)v);
    case 2:
      return (uint32_t)dpp<0x4E>((int)v);
    case 4:
      return (uint32_t)dpp<0x1B>(dpp<0x141>((int)v));
    case 8:
      return (uint32_t)dpp<0x141>(dpp<0x140>((int)v));
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

// The lanes whose index has bit b set (b a power of two), as a lane mask.
constexpr uint64_t lanes_with(int b) {
  return b == 1    ? 0xAAAAAAAAAAAAAAAAull
         : b == 2  ? 0xCCCCCCCCCCCCCCCCull
         : b == 4  ? 0xF0F0F0F0F0F0F0F0ull
         : b == 8  ? 0xFF00FF00FF00FF00ull
         : b == 16 ? 0xFFFF0000FFFF0000ull
         : b == 32 ? 0xFFFFFFFF00000000ull
                   : 0ull;
}

// Lanes l with l mod g < n, as a lane mask (g a power of two).
constexpr uint64_t lanes_mod_below(int g, int n) {
  uint64_t m = 0;
  for (int l = 0; l < kWave; l++)
    if (l % g < n) m |= 1ull << l;
  return m;
}

// True in the lanes of a lane mask.  With a compile-time mask the test needs
// no vector instruction; a comparison of the lane index is a vector compare
// whose result the compiler hoists out of every loop into a scalar register
// pair, which then has to be spilled and reloaded where registers are short.
__device__ __forceinline__ bool lane_in(uint64_t mask) {
  return __builtin_amdgcn_inverse_ballot_w64(mask);
}

// One compare-exchange step of a sorting network with the partner lane ^ j:
// lanes in the mask keep_max keep the larger of the two keys, the others
// the smaller.  One comparison; the direction is applied to its lane mask
// by a scalar xor.  Equal keys are equal values, so either choice is the
// same result.
__device__ __forceinline__ uint64_t cx64(uint64_t v, int j, uint64_t keep_max, int lane) {
  const uint64_t p = xor64(v, j, lane);
  return __builtin_amdgcn_inverse_ballot_w64(ballot(v > p) ^ keep_max) ? p : v;
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
