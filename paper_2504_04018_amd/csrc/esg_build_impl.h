// Device kernels of the index builder's insertion rounds (Alg. 3; the graph
// construction recalled in Section 2.1): occlusion pruning of each new
// point's search candidates into its forward row, and the reverse edges,
// which append to a target's row or re-prune it when it would overflow.
// The rules are the host builder's, with the same float32 distance and
// (distance, position) order, so both builders write the same rows.
#pragma once

#include "esg_search_impl.h"

namespace esgk {

struct BuildArgs {
  SearchArgs A;              // vectors (vec, d, dp) for the distance gathers
  int64_t nb;                // points of this round
  int32_t efc, R;            // candidates per point, row slots
  int32_t keycap;            // LDS keys per wave (a power of two)
  int32_t wave_lds;          // LDS bytes per wave
  const uint32_t* pts;       // [nb] positions inserted this round
  const int64_t* cand_ids;   // [nb][efc] search results (positions), -1 pad
  const float* cand_d;       // [nb][efc] their distances
  uint32_t* rows;            // [n][R] adjacency of the depth being built
  int32_t* cnt;              // [n] reverse-edge proposals per target (kept at 0 between rounds)
  const int32_t* start;      // [n] first slot of a target's proposals in srcs
  const uint32_t* srcs;      // proposals grouped by target
  const int32_t* touched;    // targets with proposals
  const int32_t* counters;   // [0] number of touched targets
};

// Ascending bitonic sort of keys[0, mp) in LDS by one wave (mp a power of
// two; every compare-exchange pair is owned by its lower index).
__device__ __forceinline__ void lds_sort_wave(uint64_t* keys, int mp, int lane) {
  for (int k = 2; k <= mp; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < mp; i += kWave) {
        const int l = i ^ j;
        if (l > i) {
          const uint64_t a = keys[i], b = keys[l];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            keys[i] = b;
            keys[l] = a;
          }
        }
      }
      wave_lds_sync();
    }
}

// Occlusion rule over keys[0, m) (ascending (distance to the base point,
// position)): walk the candidates in order and keep one unless an already
// kept neighbour s is strictly closer to it than the base point is; skip
// `self`; stop at R kept.  Realised one kept neighbour at a time: when s is
// kept, every later candidate still alive is compared with s at once (a
// gathered batch of distances) and dropped if s occludes it, which decides
// each candidate against the same kept neighbours, in the same order, as
// the sequential walk.  Bit 63 of a key marks a dropped candidate.  The
// kept positions go to kept[0, return value).
template <int G, int CPL>
__device__ int occlude_wave(const SearchArgs& A, WaveLds* L, uint64_t* keys, int m,
                            uint32_t self, int R, uint32_t* kept, int lane) {
  constexpr uint64_t kDead = 1ull << 63;
  int nk = 0, cursor = 0;
  float qr[CPL][4];
  while (nk < R) {
    int i = -1;
    for (int base = cursor; base < m; base += kWave) {
      const int j = base + lane;
      const uint64_t b = ballot(j < m && (keys[j] & kDead) == 0);
      if (b) {
        i = base + (int)__builtin_ctzll(b);
        break;
      }
    }
    if (i < 0) break;
    cursor = i + 1;
    const uint32_t s = key_pos(keys[i]);
    if (s == self) continue;
    if (lane == 0) kept[nk] = s;
    nk++;
    if (nk == R) break;
    load_query<kF32, G, CPL>(A.vec + (size_t)s * A.dp, A.d, lane, qr);
    for (int base = cursor; base < m; base += kWave) {
      const int j = base + lane;
      const uint64_t kj = j < m ? keys[j] : kKeyInf;
      const bool alive = j < m && (kj & kDead) == 0;
      const uint64_t b = ballot(alive);
      if (!b) continue;
      const int na = __popcll(b);
      if (alive) {
        const int rk = rank_below(b);
        L->ids[rk] = key_pos(kj);
        L->stage[rk] = (uint64_t)j;
      }
      wave_lds_sync();
      for (int c0 = 0; c0 < na; c0 += kBatch) {
        const int nn = na - c0 < kBatch ? na - c0 : kBatch;
        const uint32_t nid = lane < nn ? L->ids[c0 + lane] : kNoNode;
        const int jj = lane < nn ? (int)L->stage[c0 + lane] : 0;
        const float dd = batch_dist<kF32, G, CPL>(A, nid, nn, qr, L, lane);
        if (lane < nn) {
          const uint64_t kk = keys[jj];
          if (dd < key_dist(kk)) keys[jj] = kk | kDead;
        }
        wave_lds_sync();
      }
    }
  }
  wave_lds_sync();
  return nk;
}

__device__ __forceinline__ void build_wave_lds(const BuildArgs& B, WaveLds*& L, uint64_t*& keys,
                                               uint32_t*& kept) {
  extern __shared__ __align__(16) uint8_t smem[];
  uint8_t* base = smem + (size_t)(threadIdx.x >> 6) * (size_t)B.wave_lds;
  L = reinterpret_cast<WaveLds*>(base);
  keys = reinterpret_cast<uint64_t*>(base + kStageBytes);
  kept = reinterpret_cast<uint32_t*>(keys + B.keycap);
}

// Forward rows: point pts[i]'s search candidates, pruned to at most R.
template <int G, int CPL>
__global__ __launch_bounds__(256) void build_prune_kernel(BuildArgs B) {
  const int lane = lane_id();
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= B.nb) return;
  WaveLds* L;
  uint64_t* keys;
  uint32_t* kept;
  build_wave_lds(B, L, keys, kept);
  const uint32_t p = B.pts[i];
  const int64_t* ci = B.cand_ids + i * B.efc;
  const float* cd = B.cand_d + i * B.efc;
  int m = 0;
  for (int j0 = 0; j0 < B.efc; j0 += kWave) {
    const int j = j0 + lane;
    const int64_t id = j < B.efc ? ci[j] : -1;
    if (j < B.efc) keys[j] = id < 0 ? kKeyInf : make_key(cd[j], (uint32_t)id);
    m += __popcll(ballot(id >= 0));
  }
  wave_lds_sync();
  const int nk = occlude_wave<G, CPL>(B.A, L, keys, m, p, B.R, kept, lane);
  if (lane < B.R) B.rows[(size_t)p * B.R + lane] = lane < nk ? kept[lane] : kNoNode;
}

// Reverse edges, one target per wave: a row with room takes the new
// sources in increasing position order; a row that would overflow is
// rebuilt by the occlusion rule over its entries and the new sources,
// sorted by (distance to the target, position).
template <int G, int CPL>
__global__ __launch_bounds__(256) void build_reverse_kernel(BuildArgs B) {
  const int lane = lane_id();
  const int64_t nt = B.counters[0];
  WaveLds* L;
  uint64_t* keys;
  uint32_t* kept;
  build_wave_lds(B, L, keys, kept);
  const int wpb = (int)(blockDim.x >> 6);
  for (int64_t u = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); u < nt;
       u += (int64_t)gridDim.x * wpb) {
    const uint32_t c = (uint32_t)B.touched[u];
    const int cntc = B.cnt[c];
    const uint32_t* src = B.srcs + B.start[c];
    uint32_t* row = B.rows + (size_t)c * B.R;
    const uint32_t rv = lane < B.R ? row[lane] : kNoNode;
    const int len = __popcll(ballot(rv != kNoNode));
    if (len + cntc <= B.R) {
      uint64_t v = lane < cntc ? (uint64_t)src[lane] : kKeyInf;
      v = sort32(v, lane, cntc);
      if (lane < cntc) row[len + lane] = (uint32_t)v;
    } else {
      const int m = len + cntc;
      int mp = 1;
      while (mp < m) mp <<= 1;
      float qr[CPL][4];
      load_query<kF32, G, CPL>(B.A.vec + (size_t)c * B.A.dp, B.A.d, lane, qr);
      for (int c0 = 0; c0 < m; c0 += kBatch) {
        const int nn = m - c0 < kBatch ? m - c0 : kBatch;
        const int j = c0 + lane;
        const uint32_t pos = lane < nn ? (j < len ? row[j] : src[j - len]) : kNoNode;
        const float dd = batch_dist<kF32, G, CPL>(B.A, pos, nn, qr, L, lane);
        if (lane < nn) keys[j] = make_key(dd, pos);
      }
      for (int j = m + lane; j < mp; j += kWave) keys[j] = kKeyInf;
      wave_lds_sync();
      lds_sort_wave(keys, mp, lane);
      const int nk = occlude_wave<G, CPL>(B.A, L, keys, m, c, B.R, kept, lane);
      if (lane < B.R) row[lane] = lane < nk ? kept[lane] : kNoNode;
    }
    if (lane == 0) B.cnt[c] = 0;
    wave_lds_sync();
  }
}

}  // namespace esgk
