// Brute-force range scan on gfx950: bfloat16 MFMA candidates, float32 rerank.
//
// The exact answer of Def. 2.2 for a query is the top k of its range by
// the float32 canonical distance (ties by position).  The scan gets it in
// four kernels:
//  1. mfma_dist: one wave per block of 16 windows (a window is at most
//     kWin consecutive positions of one query's range; windows are sorted by
//     start so a block's windows overlap).  The wave walks the block's union
//     span in tiles of 16 positions; v_mfma_f32_16x16x32_bf16 forms the dot
//     products of 16 points with the 16 window queries (bfloat16 inputs,
//     float32 accumulation); approx = |x|^2 + |q|^2 - 2 x.q (norms in float32
//     from the float32 data) is written for every (window, position) pair
//     inside the window.
//  2. select: one wave per window keeps the 64*E smallest approx keys.
//  3. rerank: one wave per query merges its windows' lists, recomputes the
//     first m_r candidates with the float32 canonical distance and keeps the
//     top k.  The result is certified exact when the k-th float32 distance is
//     below (A - eps)(1 - g) / (1 + g), A being the (m_r+1)-th smallest approx
//     distance, eps the bound on |approx - exact| (bfloat16 rounding of x and
//     q, float32 accumulation and norms) and g a float32 relative error bound:
//     then no point outside the candidates can enter the top k.
//  4. fallback: queries that are not certified are rescanned exactly
//     (float32 canonical distances): each window's exact top k, one wave
//     per window, then one merge per query.
#pragma once

#include "esg_search_kernel.h"

namespace esgk {

constexpr int kWin = 2048;  // longest window scored by one select wave

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

struct ScanArgs {
  const float* vec;        // [n][dp] float32
  const uint16_t* vec16;   // [n][dp] bfloat16 bits
  const float* norm2;      // [n] |x|^2 in float32
  const int64_t* ext_id;   // [n]
  int64_t n;
  int32_t d, dp;
  const float* queries;    // [nq][d]
  const int64_t* l;
  const int64_t* r;
  int64_t nq;
  int32_t k, mr;           // results per query, candidates reranked
  // windows (sorted by start for the MFMA kernel)
  const int32_t* win_q;    // [nw] query of each window
  const int64_t* win_s;    // [nw] first position
  const int64_t* win_e;    // [nw] last position
  const int32_t* win_order;// [nw] windows sorted by start (mfma) ; null = identity
  const int32_t* q_win0;   // [nq] first window of each query (windows of a query are consecutive)
  const int32_t* q_nwin;   // [nq] number of windows of each query
  const int32_t* qlist;    // [nq_list] queries handled (null = all nq)
  const int32_t* n_win_dev;// device count of windows (null: use nw)
  const int32_t* n_q_dev;  // device count of listed queries (null: use nq_list)
  int64_t nw, nq_list;
  float* dist_buf;         // [nw][kWin] approx distances
  uint64_t* cand;          // [nw][64*E] selected keys per window
  int64_t cand_stride;
  // outputs
  int64_t* ids;            // [nq][k]
  float* dists;            // [nq][k]
  int32_t force_exact;     // 1: no certificate, every query is rescanned exactly
  int32_t* fb_list;        // [nq] queries that need the exact fallback
  int32_t* fb_count;       // [1]
  int32_t* certified;      // [nq] 1 when certified (optional, may be null)
  float delta_x;           // largest relative bfloat16 rounding error of the data
  float maxnorm;           // largest |x|
  float gamma;             // float32 accumulation bound (d + 4) * 2^-24
  float g_rel;             // float32 relative error bound of the canonical distance
};

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

// Non-negative float as a sortable key (negative approximations clamp to 0).
__device__ __forceinline__ uint64_t approx_key(float a, uint32_t pos) {
  return make_key(a > 0.0f ? a : 0.0f, pos);
}

// ---- 1. MFMA distances ------------------------------------------------------
template <int NK>  // dp / 32 rounded up: 32-wide K chunks
__global__ __launch_bounds__(256) void mfma_dist_kernel(ScanArgs S) {
  const int lane = lane_id();
  const int64_t nw = S.n_win_dev ? *S.n_win_dev : S.nw;
  const int64_t block = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t w0 = block * 16;
  if (w0 >= nw) return;
  const int col = lane & 15;   // window (B column) and point (A row) index in the tile
  const int grp = lane >> 4;   // K group of 8 within a 32-wide chunk
  // this lane's window (column)
  const int64_t wi = w0 + col;
  const bool wvalid = wi < nw;
  const int32_t wid = wvalid ? (S.win_order ? S.win_order[wi] : (int32_t)wi) : 0;
  const int32_t qid = wvalid ? S.win_q[wid] : 0;
  const int64_t ws = wvalid ? S.win_s[wid] : 0, we = wvalid ? S.win_e[wid] : -1;
  // query operand (B): bfloat16 of q[32c + 8*grp .. +7]
  bf16x8_t qb[NK];
  float qn = 0.0f;
  const float* q = S.queries + (int64_t)qid * S.d;
#pragma unroll
  for (int c = 0; c < NK; c++) {
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int j = 32 * c + 8 * grp + e;
      const float v = (wvalid && j < S.d) ? q[j] : 0.0f;
      qb[c][e] = __builtin_bit_cast(__bf16, f32_to_bf16_rne(v));
    }
  }
  // |q|^2 in float32 (each lane sums its 8*NK values; the 4 groups add)
  {
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < NK; c++)
#pragma unroll
      for (int e = 0; e < 8; e++) {
        const int j = 32 * c + 8 * grp + e;
        const float v = (wvalid && j < S.d) ? q[j] : 0.0f;
        s = __builtin_fmaf(v, v, s);
      }
    s += xor_f(s, 16, lane);
    s += xor_f(s, 32, lane);
    qn = s;
  }
  // union span of the block
  int64_t lo = wvalid ? ws : INT64_MAX, hi = wvalid ? we : -1;
#pragma unroll
  for (int s = 1; s < 16; s <<= 1) {
    const int64_t olo = (int64_t)(((uint64_t)xor_u32((uint32_t)(lo >> 32), s, lane) << 32) |
                                  xor_u32((uint32_t)lo, s, lane));
    const int64_t ohi = (int64_t)(((uint64_t)xor_u32((uint32_t)(hi >> 32), s, lane) << 32) |
                                  xor_u32((uint32_t)hi, s, lane));
    lo = olo < lo ? olo : lo;
    hi = ohi > hi ? ohi : hi;
  }
  lo = (int64_t)readlane64((uint64_t)lo, 0);
  hi = (int64_t)readlane64((uint64_t)hi, 0);
  if (hi < lo) return;
  // query norms of the 16 columns, for the output layout below
  const float qn_col = qn;  // lane's own column (lanes col, col+16, ... hold the same value)
  float* dbuf = S.dist_buf + (int64_t)wid * kWin;
  const uint16_t* X = S.vec16;
  for (int64_t t0 = lo & ~(int64_t)15; t0 <= hi; t0 += 16) {
    // skip tiles no window of the block touches (blocks may straddle gaps)
    const bool touch = wvalid && ws <= t0 + 15 && we >= t0;
    if (ballot(touch) == 0) {
      int64_t nxt = (wvalid && we >= t0 + 16) ? (ws > t0 + 16 ? ws : t0 + 16) : INT64_MAX;
#pragma unroll
      for (int s = 1; s < 16; s <<= 1) {
        const int64_t o = (int64_t)(((uint64_t)xor_u32((uint32_t)(nxt >> 32), s, lane) << 32) |
                                    xor_u32((uint32_t)nxt, s, lane));
        nxt = o < nxt ? o : nxt;
      }
      nxt = (int64_t)readlane64((uint64_t)nxt, 0);
      if (nxt == INT64_MAX) break;
      t0 = (nxt & ~(int64_t)15) - 16;
      continue;
    }
    // A operand: point t0 + col, dims 32c + 8*grp .. +7
    const int64_t prow = t0 + col;
    const bool prow_ok = prow < S.n;
    f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < NK; c++) {
      const int j0 = 32 * c + 8 * grp;
      uint4 raw = make_uint4(0, 0, 0, 0);
      if (prow_ok && j0 < S.dp) raw = *reinterpret_cast<const uint4*>(X + prow * S.dp + j0);
      const bf16x8_t a = __builtin_bit_cast(bf16x8_t, raw);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, qb[c], acc, 0, 0, 0);
    }
    // D layout: lane holds rows (points) 4*grp + i, column (window) col
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int64_t p = t0 + 4 * grp + i;
      if (wvalid && p >= ws && p <= we) {
        const float ap = S.norm2[p] + qn_col - 2.0f * acc[i];
        dbuf[p - ws] = ap;
      }
    }
  }
}

// ---- 2. per-window selection ----------------------------------------------------
template <int E>
__global__ __launch_bounds__(256) void select_kernel(ScanArgs S) {
  const int lane = lane_id();
  const int64_t nw = S.n_win_dev ? *S.n_win_dev : S.nw;
  const int64_t wi = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wi >= nw) return;
  const int32_t wid = S.win_order ? S.win_order[wi] : (int32_t)wi;
  const int64_t ws = S.win_s[wid], we = S.win_e[wid];
  const int w = (int)(we - ws + 1);
  const float* dbuf = S.dist_buf + (int64_t)wid * kWin;
  uint64_t L[E];
  list_clear(L);
  constexpr int cap = kWave * E;
  for (int base = 0; base < w; base += kBatch) {
    const int i = base + lane;
    uint64_t key = (lane < kBatch && i < w) ? approx_key(dbuf[i], (uint32_t)(ws + i)) : kKeyInf;
    const uint64_t worst = list_at(L, cap - 1);
    if (worst != kKeyInf && worst < key) key = kKeyInf;
    const uint64_t sm = ballot(key != kKeyInf);
    if (sm == 0) continue;
    if (__popcll(sm) <= 4) {
      for (uint64_t mm = sm; mm; mm &= mm - 1)
        list_insert(L, readlane64(key, __builtin_ctzll(mm)), cap, lane);
    } else {
      key = sort32(key, lane);
      list_merge32(L, bperm64(key, 63 - lane), cap, lane);
    }
  }
  uint64_t* out = S.cand + (int64_t)wid * S.cand_stride;
#pragma unroll
  for (int e = 0; e < E; e++) out[e * kWave + lane] = L[e];
}

// ---- 3. merge, float32 rerank, certification ----------------------------------------
template <int G32, int CPL32, int E>
__global__ __launch_bounds__(256) void rerank_kernel(ScanArgs S) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  WaveLds* Ls = reinterpret_cast<WaveLds*>(smem + (size_t)wave * kStageBytes);
  const int64_t nql = S.n_q_dev ? *S.n_q_dev : S.nq_list;
  const int64_t t = (int64_t)blockIdx.x * 4 + wave;
  if (t >= nql) return;
  const int32_t qi = S.qlist ? S.qlist[t] : (int32_t)t;
  constexpr int cap = kWave * E;
  // merge the windows' candidate lists
  uint64_t L[E];
  list_clear(L);
  const int32_t w0 = S.q_win0[qi], nwq = S.q_nwin[qi];
  for (int32_t j = 0; j < nwq; j++) {
    const uint64_t* c = S.cand + (int64_t)(w0 + j) * S.cand_stride;
    uint64_t B[E];
#pragma unroll
    for (int e = 0; e < E; e++) B[e] = c[e * kWave + lane];
    if (j == 0) {
#pragma unroll
      for (int e = 0; e < E; e++) L[e] = B[e];
    } else {
      list_merge(L, B, cap, lane);
    }
  }
  // float32 rerank of the first mr candidates
  const int mr = S.mr;
  const float* q = S.queries + (int64_t)qi * S.d;
  float qr32[CPL32][4];
  load_query<kF32, G32, CPL32>(q, S.d, lane, qr32);
  SearchArgs A;
  A.vec = S.vec;
  A.d = S.d;
  A.dp = S.dp;
  const int k = S.k;
  uint64_t R[E];
  list_clear(R);
#pragma unroll
  for (int e = 0; e < E; e++) {
#pragma unroll
    for (int s = 0; s < kWave / kBatch; s++) {
      const int base = e * kWave + s * kBatch;
      if (base >= mr) break;
      const uint64_t kq = bperm64(L[e], (s * kBatch + lane) & 63);
      const bool ok = lane < kBatch && base + lane < mr && kq != kKeyInf;
      const uint64_t okm = ballot(ok);
      const int n_new = __popcll(okm);
      if (n_new == 0) continue;
      const uint32_t nid = ok ? key_pos(kq) : kNoNode;  // ok lanes are a prefix
      const float bd = batch_dist<kF32, G32, CPL32>(A, nid, n_new, qr32, Ls, lane);
      uint64_t key = lane < n_new ? make_key(bd, nid) : kKeyInf;
      key = sort32(key, lane);
      list_merge32(R, bperm64(key, 63 - lane), k, lane);
    }
  }
  // certification
  const uint64_t kth = list_at(R, k - 1);
  const uint64_t next = mr < cap ? list_at(L, mr) : kKeyInf;  // (mr+1)-th approx key
  bool certified = true;
  if (next != kKeyInf && kth != kKeyInf) {
    // |approx - exact| <= 2 (dx + dq + dx dq) |x||q|            (bfloat16 rounding)
    //                    + gamma (2 |x||q| (1+dx)(1+dq) + |x|^2 + |q|^2)  (float32 sums)
    float qn = 0.0f, dq = 0.0f;
    for (int j = lane; j < S.d; j += kWave) {
      const float v = q[j];
      qn = __builtin_fmaf(v, v, qn);
      const float vb = __uint_as_float((uint32_t)f32_to_bf16_rne(v) << 16);
      if (v != 0.0f) dq = fmaxf(dq, fabsf(vb - v) / fabsf(v));
    }
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
      qn += xor_f(qn, s, lane);
      dq = fmaxf(dq, xor_f(dq, s, lane));
    }
    const float qnorm = __builtin_sqrtf(qn) * 1.0001f;
    const float M = S.maxnorm * 1.0001f, dx = S.delta_x;
    const float eps = 2.0f * (dx + dq + dx * dq) * M * qnorm +
                      S.gamma * (2.0f * M * qnorm * (1.0f + dx) * (1.0f + dq) + M * M + qnorm * qnorm);
    const float a_next = key_dist(next);
    const float lhs = key_dist(kth) * (1.0f + S.g_rel);
    const float rhs = (a_next - eps) * (1.0f - S.g_rel);
    certified = lhs < rhs;
  } else if (next != kKeyInf && kth == kKeyInf) {
    certified = false;  // fewer than k reranked but more points exist
  }
  if (S.force_exact) certified = false;
  if (S.certified && lane == 0) S.certified[qi] = certified ? 1 : 0;
  if (!certified) {
    if (lane == 0) {
      const int32_t slot = atomicAdd(S.fb_count, 1);
      S.fb_list[slot] = qi;
    }
    return;
  }
  int64_t* ids = S.ids + (int64_t)qi * k;
  float* dists = S.dists + (int64_t)qi * k;
#pragma unroll
  for (int e = 0; e < E; e++) {
    const int i = e * kWave + lane;
    if (i < k) {
      const uint64_t key = R[e];
      ids[i] = key == kKeyInf ? -1 : S.ext_id[key_pos(key)];
      dists[i] = key == kKeyInf ? __int_as_float(0x7F800000) : key_dist(key);
    }
  }
}

// ---- 4. exact fallback ------------------------------------------------------------
// 4a. Every window of an uncertified query gets its exact top k (float32
// canonical distances, ties by position), written over the window's
// candidate list.  All waves walk the (short) fallback list; the windows of
// one query are spread over the waves, so a wide range is rescanned by
// hundreds of waves at once.
template <int G32, int CPL32, int E>
__global__ __launch_bounds__(256) void fallback_window_kernel(ScanArgs S) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  WaveLds* Ls = reinterpret_cast<WaveLds*>(smem + (size_t)wave * kStageBytes);
  const int64_t nfb = *S.fb_count;
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave, nwaves = (int64_t)gridDim.x * 4;
  SearchArgs A;
  A.vec = S.vec;
  A.d = S.d;
  A.dp = S.dp;
  for (int64_t t = 0; t < nfb; t++) {
    const int32_t qi = S.fb_list[t];
    const int64_t w0 = S.q_win0[qi], nwq = S.q_nwin[qi];
    if (gw >= nwq) continue;
    float qr32[CPL32][4];
    load_query<kF32, G32, CPL32>(S.queries + (int64_t)qi * S.d, S.d, lane, qr32);
    for (int64_t j = gw; j < nwq; j += nwaves) {
      Part pt;
      pt.x = (uint32_t)S.win_s[w0 + j];
      pt.y = (uint32_t)S.win_e[w0 + j];
      uint64_t R[E];
      scan_leaf<G32, CPL32, E>(A, Ls, pt, S.k, qr32, R, lane);
      uint64_t* out = S.cand + (w0 + j) * S.cand_stride;
#pragma unroll
      for (int e = 0; e < E; e++) out[e * kWave + lane] = R[e];
    }
  }
}

// 4b. One wave per uncertified query merges its windows' exact lists and
// writes the top k (the top k of a union is inside the union of top k's).
template <int E>
__global__ __launch_bounds__(256) void fallback_merge_kernel(ScanArgs S) {
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  const int64_t nfb = *S.fb_count;
  const int k = S.k;
  for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < nfb; t += (int64_t)gridDim.x * 4) {
    const int32_t qi = S.fb_list[t];
    const int64_t w0 = S.q_win0[qi], nwq = S.q_nwin[qi];
    uint64_t R[E];
    list_clear(R);
    for (int64_t j = 0; j < nwq; j++) {
      const uint64_t* c = S.cand + (w0 + j) * S.cand_stride;
      uint64_t B[E];
#pragma unroll
      for (int e = 0; e < E; e++) B[e] = c[e * kWave + lane];
      list_merge(R, B, k, lane);
    }
    int64_t* ids = S.ids + (int64_t)qi * k;
    float* dists = S.dists + (int64_t)qi * k;
#pragma unroll
    for (int e = 0; e < E; e++) {
      const int i = e * kWave + lane;
      if (i < k) {
        const uint64_t key = R[e];
        ids[i] = key == kKeyInf ? -1 : S.ext_id[key_pos(key)];
        dists[i] = key == kKeyInf ? __int_as_float(0x7F800000) : key_dist(key);
      }
    }
  }
}

}  // namespace esgk
