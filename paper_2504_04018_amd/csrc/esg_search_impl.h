// Range-filtered beam search on gfx950: one wave64 per query.
//
// Per query the wave
//  1. picks at most two tree nodes with Alg. 4 (integer descent, Section 4.2),
//  2. runs Alg. 1 under POST (Sections 2.1-2.2) on each graph node, or scans
//     a leaf, and
//  3. merges the two answers (Alg. 4, last step) and writes the top k.
//
// Data layout inside the wave:
//  - P (candidates) and Q (results) are sorted ascending lists of 64-bit
//    keys (float distance bits above the position), held in registers as
//    E words per lane; element i lives in word i/64 of lane i%64.
//  - One expansion reads the adjacency row of the popped candidate (R <= 32
//    lanes x 4 B, prefetched while the previous expansion merges), tests
//    and sets the visited entries in an exact LDS hash (a global bitmap
//    takes new keys once the hash is 3/4 full), gathers the new
//    neighbours' vectors with 16-byte loads (G lanes per vector), reduces
//    each distance across its G lanes, drops keys that lose to a full Q,
//    sorts the rest (<= 32) with a bitonic network and merges them into P
//    and (the in-range ones) into Q.
//  - Merging a whole expansion at once gives the same P, Q and visited set
//    as inserting the neighbours one by one (Alg. 1 cuts Q back to m only
//    after the neighbour loop; P keeps its cand_cap best).
//
// Distances follow one fixed float32 order: each lane owns chunks t, t+G,
// ... of W consecutive dimensions (one 16-byte load), accumulates each
// squared difference with one fma, then the G lanes add pairwise
// (xor-butterfly: the adjacent-pair tree).
#pragma once

#include "esg_kernels.h"
#include "esg_wave.h"

namespace esgk {

template <int KIND>
struct Traits;
template <>
struct Traits<kF32> {
  static constexpr int W = 4;
};
template <>
struct Traits<kBF16> {
  static constexpr int W = 8;
};
template <>
struct Traits<kFP8> {
  static constexpr int W = 16;
};

struct WaveLds {
  uint64_t stage[64];
  float fstage[64];
  uint32_t ids[64];
};
static_assert(sizeof(WaveLds) == kStageBytes, "staging size");

__device__ __forceinline__ uint32_t* wave_table(WaveLds* L) {
  return reinterpret_cast<uint32_t*>(L + 1);
}

// ---- distances ------------------------------------------------------------

template <int KIND>
__device__ __forceinline__ uint4 load_chunk(const SearchArgs& A, uint32_t id, int ch) {
  // row offset as one 32 x 32 -> 64-bit product (dp is positive)
  const uint64_t row = (uint64_t)id * (uint32_t)A.dp;
  const uint4* p;
  if constexpr (KIND == kF32)
    p = reinterpret_cast<const uint4*>(A.vec + row) + ch;
  else if constexpr (KIND == kBF16)
    p = reinterpret_cast<const uint4*>(A.vec16 + row) + ch;
  else
    p = reinterpret_cast<const uint4*>(A.vec8 + row) + ch;
  return *p;
}

__device__ __forceinline__ float sqacc(float x, float q, float acc) {
  float delta = x - q;
  return __builtin_fmaf(delta, delta, acc);
}

template <int KIND>
__device__ __forceinline__ float chunk_acc(const uint4& raw, const float* qc, float scale, float acc) {
  const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
  if constexpr (KIND == kF32) {
#pragma unroll
    for (int e = 0; e < 4; e++) acc = sqacc(__uint_as_float(w[e]), qc[e], acc);
  } else if constexpr (KIND == kBF16) {
#pragma unroll
    for (int e = 0; e < 8; e++) {
      uint32_t h = (e & 1) ? (w[e >> 1] & 0xFFFF0000u) : (w[e >> 1] << 16);
      acc = sqacc(__uint_as_float(h), qc[e], acc);
    }
  } else {
    // gfx950 converts two OCP E4M3 bytes to float32 per instruction (exact)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[j], false);
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[j], true);
      acc = sqacc(scale * lo[0], qc[4 * j + 0], acc);
      acc = sqacc(scale * lo[1], qc[4 * j + 1], acc);
      acc = sqacc(scale * hi[0], qc[4 * j + 2], acc);
      acc = sqacc(scale * hi[1], qc[4 * j + 3], acc);
    }
  }
  return acc;
}


template <int KIND, int G, int CPL>
__device__ __forceinline__ void load_query(const float* q, int d, int lane,
                                           float (&qr)[CPL][Traits<KIND>::W]) {
  constexpr int W = Traits<KIND>::W;
  const int t = lane % G;
#pragma unroll
  for (int c = 0; c < CPL; c++)
#pragma unroll
    for (int e = 0; e < W; e++) {
      int j = (t + c * G) * W + e;
      qr[c][e] = j < d ? q[j] : 0.0f;
    }
}

// Distances of up to 32 vectors whose positions sit in lanes 0..n_new-1 of
// `nid`.  Returns lane j's distance (j < n_new).
template <int KIND, int G, int CPL, int RFMAX = 8, int TGMAX = (KIND == kF32 ? 8 : 1)>
__device__ __forceinline__ float batch_dist(const SearchArgs& A, uint32_t nid, int n_new,
                                            const float (&qr)[CPL][Traits<KIND>::W], WaveLds* L,
                                            int lane) {
  constexpr int W = Traits<KIND>::W;
  constexpr int VPG = (kWave / G) < kBatch ? (kWave / G) : kBatch;  // vectors per round
  constexpr int NR = (kBatch + VPG - 1) / VPG;                       // rounds for a full batch
  // fp8 rows that take a whole wave with one chunk per lane (768 and 1,024
  // values) keep 12 rounds in flight: a hop's dozen new vectors then need
  // one memory round trip instead of two, within the same two waves per
  // SIMD (measured 5 % faster at d = 768)
  constexpr int RFK = (KIND == kFP8 && G == kWave && CPL == 1 && RFMAX == 8) ? 12 : RFMAX;
  constexpr int RF0 = RFK / CPL;
  constexpr int RF = RF0 < 1 ? 1 : (RF0 > NR ? NR : RF0);            // rounds in flight
  const int grp = lane / G, t = lane % G;
  const int C = (A.d + W - 1) / W;
#pragma unroll
  for (int r0 = 0; r0 < NR; r0 += RF) {
    if (r0 * VPG >= n_new) break;
    uint4 raw[RF][CPL];
    float sc[RF];
#pragma unroll
    for (int rr = 0; rr < RF; rr++) {
      const int slot = (r0 + rr) * VPG + grp;
      const uint32_t id = bperm(nid, slot & 63);
      const bool ok = grp < VPG && slot < n_new;
#pragma unroll
      for (int c = 0; c < CPL; c++) {
        const int ch = t + c * G;
        raw[rr][c] = (ok && ch < C) ? load_chunk<KIND>(A, id, ch) : make_uint4(0, 0, 0, 0);
      }
      if constexpr (KIND == kFP8) sc[rr] = ok ? A.scale8[id] : 0.0f;
      else sc[rr] = 1.0f;
    }
    // Reduce TG rounds at a time across the G lanes of a vector: at the step
    // with stride s < TG, the pair (t, t^s) adds its partial sums, lane t
    // keeping one half of the rounds and t^s the other, so TG-1 exchanges
    // replace TG*log2(TG) (a reduce-scatter); the remaining strides are a
    // plain butterfly.  Every sum is still formed by the adjacent-pair tree
    // (stride 1 first), so the result is bit-identical to reducing each
    // round alone.  Lane t ends with round g0 + r(t), r(t) = sum_j
    // bit_j(t) * TG/2^(j+1).
    constexpr int TG = RF < TGMAX ? RF : TGMAX;
#pragma unroll
    for (int g0 = 0; g0 < RF; g0 += TG) {
      if ((r0 + g0) * VPG >= n_new) break;    // only occupied groups are reduced
      float acc[TG];
#pragma unroll
      for (int rr = 0; rr < TG; rr++) {
        acc[rr] = 0.0f;
#pragma unroll
        for (int c = 0; c < CPL; c++)
          acc[rr] = chunk_acc<KIND>(raw[g0 + rr][c], qr[c], sc[g0 + rr], acc[rr]);
      }
      int nv = TG;
#pragma unroll
      for (int s = 1; s < TG; s <<= 1) {
        const bool upper = lane_in(lanes_with(s));
        nv >>= 1;
#pragma unroll
        for (int i = 0; i < TG / 2; i++) {
          if (i < nv) {
            const float lo = acc[i], hi = acc[i + nv];
            const float keep = upper ? hi : lo, give = upper ? lo : hi;
            acc[i] = keep + xor_f(give, s, lane);
          }
        }
      }
#pragma unroll
      for (int s = TG; s < G; s <<= 1) acc[0] = acc[0] + xor_f(acc[0], s, lane);
      constexpr uint64_t kLead = lanes_mod_below(G, TG);   // the lanes with t < TG
      if (lane_in(kLead)) {
        int r = 0;
#pragma unroll
        for (int s = 1, h = TG >> 1; s < TG; s <<= 1, h >>= 1) r += (t & s) ? h : 0;
        const int slot = (r0 + g0 + r) * VPG + grp;
        if (grp < VPG && slot < n_new) L->fstage[slot] = acc[0];
      }
    }
  }
  wave_lds_sync();
  return lane < n_new ? L->fstage[lane] : 0.0f;
}

// ---- ordered lists ------------------------------------------------------------

// Ascending sort of the 32 keys in lanes 0..31 (bitonic network), of which
// lanes n..31 hold +inf.  After the stage that sorts runs of k lanes, lanes
// 0..k-1 form an ascending run; once k >= n that run holds every finite key
// and the later stages would only move +inf keys, so they are skipped.
__device__ __forceinline__ uint64_t sort32(uint64_t v, int lane, int n = 32) {
  n = __builtin_amdgcn_readfirstlane(n);     // the same in every lane
#pragma unroll
  for (int k = 2; k <= 32; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j >= 1; j >>= 1) {
      // a lane keeps the larger key when exactly one of its bits j, k is set
      v = cx64(v, j, lanes_with(j) ^ lanes_with(k), lane);
    }
    if (k >= n) break;
  }
  return v;
}

// Sorts a bitonic list of 64*E keys ascending, then drops elements >= cap.
template <int E>
__device__ __forceinline__ void bitonic_finish(uint64_t (&L)[E], int cap, int lane) {
#pragma unroll
  for (int s = E / 2; s >= 1; s >>= 1) {
#pragma unroll
    for (int e = 0; e < E; e++) {
      if ((e & s) == 0) {
        uint64_t lo = kmin(L[e], L[e + s]), hi = kmax(L[e], L[e + s]);
        L[e] = lo;
        L[e + s] = hi;
      }
    }
  }
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
#pragma unroll
    for (int e = 0; e < E; e++) {
      L[e] = cx64(L[e], s, lanes_with(s), lane);
    }
  }
#pragma unroll
  for (int e = 0; e < E; e++)
    if (e * kWave + lane >= cap) L[e] = kKeyInf;
}

// Merges up to 32 sorted keys into the sorted list; `brev` holds them
// reversed in lanes 32..63 (lane 63-j = j-th smallest) and +inf elsewhere.
template <int E>
__device__ __forceinline__ void list_merge32(uint64_t (&L)[E], uint64_t brev, int cap, int lane) {
  L[E - 1] = kmin(L[E - 1], brev);
  bitonic_finish<E>(L, cap, lane);
}

// A one-register list that keeps at most 32 keys (lanes 32..63 hold +inf)
// takes up to 32 sorted keys `rev` given reversed in lanes 0..31 (lane 31-j
// = j-th smallest, +inf elsewhere) within the low half wave: lane i <
// 32 holding min(L[i], rev[i]) is a bitonic sequence of the 32 smallest keys
// of both, which five half-wave steps sort; the cross-half step of the full
// merge is not needed.
__device__ __forceinline__ void merge_low32(uint64_t& L, uint64_t rev, int cap, int lane) {
  L = kmin(L, rev);
#pragma unroll
  for (int s = 16; s >= 1; s >>= 1) L = cx64(L, s, lanes_with(s), lane);
  if (lane >= cap) L = kKeyInf;
}

// Merges up to 32 keys sorted ascending in lanes 0..31 (+inf elsewhere)
// into the sorted list.
template <int E>
__device__ __forceinline__ void merge_sorted32(uint64_t (&L)[E], uint64_t key, int cap, int lane) {
  if (E == 1 && cap <= 32)
    merge_low32(L[0], bperm64(key, (31 - lane) & 63), cap, lane);
  else
    list_merge32(L, bperm64(key, 63 - lane), cap, lane);
}

// Merges two sorted lists of the same shape into the first.
template <int E>
__device__ __forceinline__ void list_merge(uint64_t (&A)[E], const uint64_t (&B)[E], int cap,
                                           int lane) {
#pragma unroll
  for (int e = 0; e < E; e++) A[e] = kmin(A[e], bperm64(B[E - 1 - e], 63 - lane));
  bitonic_finish<E>(A, cap, lane);
}

// Removes element 0.
template <int E>
__device__ __forceinline__ void list_pop(uint64_t (&L)[E], int lane) {
#pragma unroll
  for (int e = 0; e < E; e++) {
    uint64_t nxt = (e + 1 < E) ? readlane64(L[e + 1 < E ? e + 1 : e], 0) : kKeyInf;
    uint64_t sh = next_lane64(L[e]);
    L[e] = lane_in(1ull << 63) ? nxt : sh;
  }
}

// Inserts one key into the sorted list (dropped when its rank is >= cap).
template <int E>
__device__ __forceinline__ void list_insert(uint64_t (&L)[E], uint64_t key, int cap, int lane) {
  int rank = 0;
#pragma unroll
  for (int e = 0; e < E; e++) rank += __popcll(ballot(L[e] < key));
  if (rank >= cap) return;
  uint64_t carry = kKeyInf;
#pragma unroll
  for (int e = 0; e < E; e++) {
    const uint64_t last = readlane64(L[e], 63);
    uint64_t prev = prev_lane64(L[e]);
    prev = lane_in(1ull) ? carry : prev;
    const int i = e * kWave + lane;
    L[e] = i < rank ? L[e] : (i == rank ? key : prev);
    if (i >= cap) L[e] = kKeyInf;
    carry = last;
  }
}

template <int E>
__device__ __forceinline__ uint64_t list_at(const uint64_t (&L)[E], int i) {
  uint64_t v = kKeyInf;
#pragma unroll
  for (int e = 0; e < E; e++)
    if (e == i / kWave) v = readlane64(L[e], i % kWave);
  return v;
}

template <int E>
__device__ __forceinline__ void list_clear(uint64_t (&L)[E]) {
#pragma unroll
  for (int e = 0; e < E; e++) L[e] = kKeyInf;
}

// ---- visited set ------------------------------------------------------------
//
// Exact visited set of one graph part [a,b], in LDS with 16-bit slots.
// A point v has the node-local key k = v - a (< 2^kb, kb = bits of the node
// size, at least log2 T).  A bijection f on kb bits (odd multiply, then an
// xor-shift) maps k to f(k); its top log2(T) bits give the home slot and
// its low rb = kb - log2(T) <= 12 bits are stored, so (home, stored bits)
// identify k.  A slot holds 0 (empty) or 0x8000 | j << 12 | low bits, where
// j < 8 is the distance from the home slot (linear probing).  A key whose
// 8 probe slots are all taken goes to a per-wave bitmap in global memory
// over [a,b]; a lookup that meets 8 taken slots without a match consults
// the bitmap.  Slots are never freed, so both structures stay exact.
//
// The bitmap is all zero between parts: each spilled key's word index is
// appended to a per-wave log, and at the end of the part exactly those
// words are cleared (the whole [a,b] span only if the log overflowed).  A
// part that never spills writes nothing to global memory for its visited
// set.

constexpr int kSpillLog = 4096;   // logged bitmap words per wave slot

struct Visited {
  uint32_t* table;   // T/2 words of two 16-bit slots
  uint32_t* bm;      // spill bitmap of this wave slot, indexed by position - a; its
                     // log (kSpillLog words set during the current part) follows at
                     // bm + spill_words
  uint32_t a, b;
  uint32_t kb_mask;  // 2^kb - 1
  int kb, shift;     // shift = kb - log2(T) (stored low bits)
  int nlog;          // keys spilled in the current part (wave-uniform)
};

__device__ __forceinline__ uint32_t vkey_mix(uint32_t k, const Visited& V) {
  uint32_t x = (k * 0x9E3779B1u) & V.kb_mask;
  return x ^ (x >> ((V.kb + 1) >> 1));
}

// End of a part: clears the bitmap words its spilled keys set, leaving the
// bitmap all zero for the next part.
__device__ __forceinline__ void visited_finish(const SearchArgs& A, Visited& V, int lane) {
  if (V.nlog == 0) return;
  __threadfence();   // every lane's log entries and bitmap updates are visible
  if (V.nlog <= kSpillLog) {
    const uint32_t* log = V.bm + A.spill_words;
    for (int i = lane; i < V.nlog; i += kWave) V.bm[log[i]] = 0u;
  } else {
    const uint32_t words = ((V.b - V.a) >> 5) + 1u;
    for (uint32_t i = (uint32_t)lane; i < words; i += kWave) V.bm[i] = 0u;
  }
  __threadfence();   // the clears land before the next part's updates
  V.nlog = 0;
}

// Test-and-set of v for active lanes; true when v was not visited before.
__device__ __forceinline__ bool visit(const SearchArgs& A, Visited& V, uint32_t v, bool active,
                                      int lane) {
  bool is_new = false, overflow = false;
  if (active) {
    const uint32_t x = vkey_mix(v - V.a, V);
    const uint32_t home = x >> V.shift;
    const uint32_t low = x & ((1u << V.shift) - 1u);
    const uint32_t tmask = (uint32_t)A.hash_cap - 1u;
    overflow = true;
    for (uint32_t j = 0; j < 8u; j++) {
      const uint32_t s = (home + j) & tmask;
      const uint32_t want = 0x8000u | (j << 12) | low;
      // one read of the slot's 32-bit word; an empty slot is claimed with a
      // CAS on that word (another lane may take either half meanwhile)
      uint32_t* word = V.table + (s >> 1);
      const uint32_t sh = (s & 1u) * 16u;
      uint32_t old = *word;
      uint32_t e = (old >> sh) & 0xFFFFu;
      while (e == 0u) {
        const uint32_t got = atomicCAS(word, old, old | (want << sh));
        if (got == old) break;
        old = got;
        e = (old >> sh) & 0xFFFFu;
      }
      if (e == 0u) { is_new = true; overflow = false; break; }
      if (e == want) { overflow = false; break; }   // already visited
    }
  }
  const uint64_t om = ballot(overflow);
  if (om != 0) {
    if (overflow) {
      const uint32_t off = v - V.a;
      const uint32_t bit = 1u << (off & 31u);
      is_new = (atomicOr(&V.bm[off >> 5], bit) & bit) == 0u;
      const int at = V.nlog + rank_below(om);
      if (at < kSpillLog) V.bm[A.spill_words + at] = off >> 5;
    }
    V.nlog += __popcll(om);
  }
  return is_new;
}

__device__ __forceinline__ void visited_reset(const SearchArgs& A, Visited& V, uint32_t a,
                                              uint32_t b, int lane) {
  V.a = a;
  V.b = b;
  int kb = 32 - __clz(b - a);                 // bits of the largest local key
  const int tbits = 31 - __clz((uint32_t)A.hash_cap);
  if (kb < tbits) kb = tbits;
  V.kb = kb;
  V.kb_mask = kb >= 32 ? 0xFFFFFFFFu : ((1u << kb) - 1u);
  V.shift = kb - tbits;
  V.nlog = 0;
  uint4* t4 = reinterpret_cast<uint4*>(V.table);
  for (int i = lane; i < A.hash_cap / 8; i += kWave) t4[i] = make_uint4(0, 0, 0, 0);
  wave_lds_sync();
}

// ---- parts ----------------------------------------------------------------------

struct Part {
  int32_t kind;  // 1 graph, 2 scan
  int32_t depth;
  int64_t heap;
  uint32_t a, b, x, y;
};

// One descent of Alg. 4 from node (a,b) with part (x,y): follows the single
// child that holds the part until a leaf or an elastic node is reached, or
// (when allow_split) until the part straddles two children, in which case
// the two pieces are returned in `it`/`right` with split = true.  Node
// [a,b] of L points has `fanout` children, child j starting at
// a + ceil(jL/fanout), so position p lies in child floor(fanout (p-a) / L);
// child j of node h is numbered fanout (h-1) + 2 + j.  A part that is not
// elastic at c = 1/fanout never straddles three children (the middle one
// would hold >= L/fanout of its points: Lemma 4.3); false is returned if it
// does, or if a piece of a split would straddle again.
struct Desc {
  int64_t a, b, x, y, heap;
  int32_t depth;
};

__device__ __forceinline__ int64_t child_begin(int64_t a, int64_t L, int32_t f, int64_t j) {
  if (f == 2) return a + ((j * L + 1) >> 1);
  return a + (j * L + f - 1) / f;
}

__device__ __forceinline__ bool descend(Desc& it, int64_t leaf, int32_t c_den, int32_t fanout,
                                        bool allow_split, Desc& right, bool& split) {
  split = false;
  for (int guard = 0; guard < 64; guard++) {
    const int64_t L = it.b - it.a + 1;
    const bool is_leaf = it.b - it.a < leaf;
    const bool elastic = !is_leaf && (int64_t)c_den * (it.y - it.x + 1) >= L;
    if (is_leaf || elastic) return true;
    int64_t jx, jy;
    if (fanout == 2) {                      // Alg. 4's split at floor((a+b)/2), no division
      const int64_t mid = (it.a + it.b) >> 1;
      jx = it.x > mid;
      jy = it.y > mid;
    } else {
      jx = (int64_t)fanout * (it.x - it.a) / L;
      jy = (int64_t)fanout * (it.y - it.a) / L;
    }
    const int64_t h0 = (int64_t)fanout * (it.heap - 1) + 2;
    const int64_t s0 = child_begin(it.a, L, fanout, jx), s1 = child_begin(it.a, L, fanout, jx + 1);
    if (jy == jx) {
      it = {s0, s1 - 1, it.x, it.y, h0 + jx, it.depth + 1};
      continue;
    }
    if (jy != jx + 1 || !allow_split) return false;
    const int64_t s2 = child_begin(it.a, L, fanout, jx + 2);
    right = {s1, s2 - 1, s1, it.y, h0 + jx + 1, it.depth + 1};
    it = {s0, s1 - 1, it.x, s1 - 1, h0 + jx, it.depth + 1};
    split = true;
    return true;
  }
  return false;
}

__device__ __forceinline__ Part to_part(const Desc& it, int64_t leaf) {
  return {it.b - it.a < leaf ? 2 : 1, it.depth, it.heap, (uint32_t)it.a, (uint32_t)it.b,
          (uint32_t)it.x, (uint32_t)it.y};
}

// Half-bounded index (Section 4.1): the tightest recorded prefix
// [0, s - 1] holding [0, rq] (ratio >= 1/B by Lemma 4.1), or for lq > 0 and
// rq = n - 1 the tightest suffix [n - s, n - 1] holding [lq, n - 1]; a
// range with both ends inside takes whichever covers it with the larger
// ratio (the prefix on a tie).  Sizes s_0 = n, s_{i+1} = ceil(s_i / B);
// depth i (prefix) or K + i (suffix) for the K sizes with a graph, node
// number depth + 1; a size without a graph (s - 1 < leaf) is scanned.
__device__ __forceinline__ Part select_chain(int64_t n, int64_t leaf, int32_t B, int64_t lq,
                                             int64_t rq) {
  int64_t sp = n, ip = 0, ss = n, is = 0, K = 0;
  for (int64_t s = n; s - 1 >= leaf; s = (s + B - 1) / B) {
    K++;
    if (s == 1) break;
  }
  for (;;) {
    const int64_t nx = (sp + B - 1) / B;
    if (nx == sp || nx < rq + 1) break;
    sp = nx;
    ip++;
  }
  for (;;) {
    const int64_t nx = (ss + B - 1) / B;
    if (nx == ss || nx < n - lq) break;
    ss = nx;
    is++;
  }
  const bool pre = lq == 0 ? true : (rq == n - 1 ? false : ss >= sp);
  const int64_t size = pre ? sp : ss;
  Part p;
  p.a = (uint32_t)(pre ? 0 : n - ss);
  p.b = (uint32_t)(pre ? sp - 1 : n - 1);
  p.x = (uint32_t)lq;
  p.y = (uint32_t)rq;
  if (size - 1 < leaf) {
    p.kind = 2;
    p.depth = -1;
    p.heap = 0;
  } else {
    p.kind = 1;
    p.depth = (int32_t)(pre ? ip : K + is);
    p.heap = p.depth + 1;
  }
  return p;
}

// Alg. 4: at most two parts (Lemma 4.2 at fanout 2, Lemma 4.3 at fanout f
// with c = 1/f).  Returns the count (or -1 if the descent would emit more:
// never when c_den >= fanout, which the loader enforces) and part `which`
// (0 or 1) in `out`.  The search recomputes the descent for each part (a few
// scalar steps) so that no part record has to be kept in memory.  A chain
// index gives one part (select_chain).
__device__ __forceinline__ int select_parts(const SearchArgs& A, int64_t lq, int64_t rq, int which,
                                            Part& out) {
  const int64_t n = A.n, leaf = A.leaf;
  const int32_t c_den = A.c_den, fanout = A.fanout;
  if (A.layout == 1) {
    out = select_chain(n, leaf, fanout, lq, rq);
    return 1;
  }
  Desc it = {0, n - 1, lq, rq, 1, 0}, right = it, dummy = it;
  bool split = false, s2 = false;
  if (!descend(it, leaf, c_den, fanout, true, right, split)) return -1;
  if (!split) {
    out = to_part(it, leaf);
    return 1;
  }
  if (!descend(it, leaf, c_den, fanout, false, dummy, s2)) return -1;
  if (!descend(right, leaf, c_den, fanout, false, dummy, s2)) return -1;
  if (which == 1) it = right;
  out = to_part(it, leaf);
  return 2;
}

}  // namespace esgk
