// Brute-force range scan on gfx950: bfloat16 MFMA candidates, float32 rerank.
//
// The exact answer of Def. 2.2 for a query is the top k of its range by
// the float32 canonical distance (ties by position).  The scan gets it in
// three steps:
//  1. scan_select: a query range is cut into windows of at most kWin
//     consecutive positions, and the windows of the batch are sorted by
//     start.  One workgroup (4 waves) takes 64 consecutive windows, 16 per
//     wave, and walks the union of their spans in tiles of TP positions: the
//     tile's bfloat16 vectors and norms are staged once in LDS for all 64
//     windows, v_mfma_f32_16x16x32_bf16 forms the dot products of 16 points
//     with a wave's 16 window queries (float32 accumulation), and
//     approx = |x|^2 + |q|^2 - 2 x.q.  Each window keeps its 64E smallest
//     approx values: a value below the window's current bound is appended to
//     the window's LDS buffer, and a full buffer is merged into the window's
//     sorted list (registers, bitonic) which lowers the bound.  Values are
//     32-bit keys: the approx bits with their low 11 mantissa bits replaced
//     by the offset in the window, so a key never exceeds the float it
//     came from (truncation toward zero keeps the certificate below
//     conservative).  Each window writes its list.
//  2. rerank: one wave per query merges its windows' lists, recomputes the
//     first m_r candidates with the float32 canonical distance and keeps the
//     top k.  The result is certified exact when the k-th float32 distance is
//     below (A - eps)(1 - g) / (1 + g), A being the value of the (m_r+1)-th
//     smallest key (no unreranked point has a smaller approx), eps the bound
//     on |approx - exact| (bfloat16 rounding of x and q, float32
//     accumulation and norms) and g a float32 relative error bound: then no
//     point outside the candidates can enter the top k.
//  3. fallback: queries that are not certified are rescanned exactly
//     (float32 canonical distances): each window's exact top k, one wave
//     per window, then one merge per query.
#pragma once

#include "esg_search_kernel.h"

namespace esgk {

constexpr int kWin = 2048;        // longest window; offsets fit the key's 11 low bits
constexpr int kScanWinPerWave = 16;
constexpr int kScanBuf = 128;     // LDS candidate buffer per window

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

struct ScanArgs {
  const float* vec;        // [n][dp] float32
  const uint16_t* vec16;   // [n][dp] bfloat16 bits
  const float* norm2;      // [n] |x|^2 in float32
  const int64_t* ext_id;   // [n]
  int64_t n;
  int32_t d, dp;
  int32_t dq;              // values per query row (<= d; the rest of a query reads as 0)
  const float* queries;    // [nq][dq]
  const int64_t* l;
  const int64_t* r;
  int64_t nq;
  int32_t k, mr;           // results per query, candidates reranked
  // windows (sorted by start for the MFMA kernel)
  int32_t* win_q;          // [nw] query of each window
  int64_t* win_s;          // [nw] first position
  int64_t* win_e;          // [nw] last position
  const int32_t* win_order;// [nw] windows sorted by start (mfma) ; null = identity
  const int32_t* q_win0;   // [nq] first window of each query (windows of a query are consecutive)
  const int32_t* q_nwin;   // [nq] number of windows of each query
  const int32_t* qlist;    // [nq_list] queries handled (null = all nq)
  const int32_t* n_win_dev;// device count of windows (null: use nw)
  const int32_t* n_q_dev;  // device count of listed queries (null: use nq_list)
  int64_t nw, nq_list;
  uint64_t* cand;          // [nw][cand_stride]: 64E 32-bit keys of the MFMA pass, or the
                           // exact 64-bit keys of the fallback
  int64_t cand_stride;     // in 64-bit slots, >= 64E
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

// Window key: approx (negative values clamp to 0) with the low 11 mantissa
// bits replaced by the offset in the window.  Its value as a float is <= the
// approx.
__device__ __forceinline__ uint32_t win_key(float a, uint32_t off) {
  return ((__float_as_uint(a > 0.0f ? a : 0.0f)) & ~0x7FFu) | off;
}
// The 64-bit candidate key (truncated approx bits, position) of a window key.
__device__ __forceinline__ uint64_t cand_key(uint32_t wk, int64_t ws) {
  return wk == 0xFFFFFFFFu ? kKeyInf
                           : ((uint64_t)(wk & ~0x7FFu) << 32) | (uint64_t)(ws + (wk & 0x7FFu));
}

// ---- 32-bit ordered lists across a wave (element i: word i/64, lane i%64) ----

__device__ __forceinline__ uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t umax32(uint32_t a, uint32_t b) { return a < b ? b : a; }

// Ascending bitonic sort of one key per lane.
__device__ __forceinline__ uint32_t sort64_u32(uint32_t v, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j >= 1; j >>= 1) {
      const uint32_t p = xor_u32(v, j, lane);
      const bool up = (lane & k) == 0;
      const bool lower = (lane & j) == 0;
      v = (lower == up) ? umin32(v, p) : umax32(v, p);
    }
  }
  return v;
}

// Keeps the 64E smallest of the sorted list L and the sorted batch b (one
// key per lane): min against the reversed batch, then a bitonic finish.
template <int E>
__device__ __forceinline__ void merge64_u32(uint32_t (&L)[E], uint32_t b, int lane) {
  L[E - 1] = umin32(L[E - 1], bperm(b, 63 - lane));
#pragma unroll
  for (int s = E / 2; s >= 1; s >>= 1) {
#pragma unroll
    for (int e = 0; e < E; e++) {
      if ((e & s) == 0) {
        const uint32_t lo = umin32(L[e], L[e + s]), hi = umax32(L[e], L[e + s]);
        L[e] = lo;
        L[e + s] = hi;
      }
    }
  }
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
#pragma unroll
    for (int e = 0; e < E; e++) {
      const uint32_t p = xor_u32(L[e], s, lane);
      L[e] = (lane & s) ? umax32(L[e], p) : umin32(L[e], p);
    }
  }
}

// ---- 1. MFMA distances and per-window selection --------------------------------------
template <int NK, int E, int TP, int DP>
__global__ __launch_bounds__(256) void scan_select_kernel(ScanArgs S) {
  constexpr int ROW = DP + 8;                  // padded LDS row (bf16 elements)
  constexpr int NWG = 4 * kScanWinPerWave;     // windows per workgroup
  __shared__ __align__(16) uint16_t tile[TP * ROW];
  __shared__ float tnorm[TP];
  constexpr int BUF = DP >= 1024 ? 96 : kScanBuf;   // keeps the LDS footprint under 64 KB
  __shared__ uint32_t buf[4][kScanWinPerWave][BUF];
  __shared__ int32_t cnt[4][kScanWinPerWave];
  __shared__ int64_t span[4][2];
  const int lane = lane_id();
  const int wave = (int)(threadIdx.x >> 6);
  const int64_t nw = S.n_win_dev ? *S.n_win_dev : S.nw;
  const int64_t wbase = (int64_t)blockIdx.x * NWG;
  if (wbase >= nw) return;                     // uniform over the workgroup
  const int col = lane & 15;   // window (B column) and point (A row) index in the tile
  const int grp = lane >> 4;   // K group of 8 within a 32-wide chunk
  const int64_t wi = wbase + wave * kScanWinPerWave + col;
  const bool wvalid = wi < nw;
  const int32_t wid = wvalid ? (S.win_order ? S.win_order[wi] : (int32_t)wi) : 0;
  const int32_t qid = wvalid ? S.win_q[wid] : 0;
  const int64_t ws = wvalid ? S.win_s[wid] : 0, we = wvalid ? S.win_e[wid] : -1;
  // query operand (B): bfloat16 of q[32c + 8*grp .. +7]; |q|^2 in float32
  bf16x8_t qb[NK];
  const float* q = S.queries + (int64_t)qid * S.dq;
  float qn = 0.0f;
#pragma unroll
  for (int c = 0; c < NK; c++) {
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int j = 32 * c + 8 * grp + e;
      const float v = (wvalid && j < S.dq) ? q[j] : 0.0f;
      qb[c][e] = __builtin_bit_cast(__bf16, f32_to_bf16_rne(v));
      qn = __builtin_fmaf(v, v, qn);
    }
  }
  qn += xor_f(qn, 16, lane);
  qn += xor_f(qn, 32, lane);
  // workgroup span: each wave reduces its 16 windows, then the 4 waves'
  int64_t wlo = wvalid ? ws : INT64_MAX, whi = wvalid ? we : -1;
#pragma unroll
  for (int s = 1; s < 16; s <<= 1) {
    const int64_t olo = (int64_t)(((uint64_t)xor_u32((uint32_t)(wlo >> 32), s, lane) << 32) |
                                  xor_u32((uint32_t)wlo, s, lane));
    const int64_t ohi = (int64_t)(((uint64_t)xor_u32((uint32_t)(whi >> 32), s, lane) << 32) |
                                  xor_u32((uint32_t)whi, s, lane));
    wlo = olo < wlo ? olo : wlo;
    whi = ohi > whi ? ohi : whi;
  }
  if (lane == 0) {
    span[wave][0] = wlo;
    span[wave][1] = whi;
  }
  if (threadIdx.x < 4 * kScanWinPerWave) (&cnt[0][0])[threadIdx.x] = 0;
  __syncthreads();
  int64_t lo = span[0][0], hi = span[0][1];
#pragma unroll
  for (int v = 1; v < 4; v++) {
    lo = span[v][0] < lo ? span[v][0] : lo;
    hi = span[v][1] > hi ? span[v][1] : hi;
  }
  uint32_t L[kScanWinPerWave][E];
#pragma unroll
  for (int w = 0; w < kScanWinPerWave; w++)
#pragma unroll
    for (int e = 0; e < E; e++) L[w][e] = 0xFFFFFFFFu;
  uint32_t tau = 0xFFFFFFFFu;                  // this lane's window: keys below enter its buffer
  int32_t* mycnt = &cnt[wave][col];
  uint32_t* mybuf = buf[wave][col];

  // merges the buffers of the windows in `need` into their lists
  auto flush = [&](uint32_t need) {
#pragma unroll
    for (int w = 0; w < kScanWinPerWave; w++) {
      if (need & (1u << w)) {
        const int c = cnt[wave][w];
        for (int b0 = 0; b0 < c; b0 += 64) {
          uint32_t v = b0 + lane < c ? buf[wave][w][b0 + lane] : 0xFFFFFFFFu;
          v = sort64_u32(v, lane);
          merge64_u32<E>(L[w], v, lane);
        }
        const uint32_t bound = readlane(L[w][E - 1], 63);
        if (col == w) tau = bound;
      }
    }
    wave_lds_sync();
    if (lane < kScanWinPerWave && (need & (1u << lane))) cnt[wave][lane] = 0;
    wave_lds_sync();
  };

  for (int64_t t0 = lo & ~(int64_t)(TP - 1); t0 <= hi; t0 += TP) {
    // skip tiles no window of the workgroup touches
    const bool touch = wvalid && ws <= t0 + TP - 1 && we >= t0;
    if (!__syncthreads_or(touch)) continue;
    // stage the tile's vectors and norms
    constexpr int CH = DP / 8;                 // 16-byte chunks per row
    for (int u = (int)threadIdx.x; u < TP * CH; u += 256) {
      const int row = u / CH, ch = u % CH;
      const int64_t p = t0 + row;
      uint4 v = make_uint4(0, 0, 0, 0);   // chunks past the index's row stay zero
      if (p < S.n && ch * 8 < S.dp) v = *reinterpret_cast<const uint4*>(S.vec16 + p * S.dp + ch * 8);
      *reinterpret_cast<uint4*>(&tile[row * ROW + ch * 8]) = v;
    }
    if (threadIdx.x < TP) {
      const int64_t p = t0 + threadIdx.x;
      tnorm[threadIdx.x] = p < S.n ? S.norm2[p] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int sub = 0; sub < TP / 16; sub++) {
      f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int c = 0; c < NK; c++) {
        const int j0 = 32 * c + 8 * grp;
        uint4 raw = make_uint4(0, 0, 0, 0);
        if (j0 < DP) raw = *reinterpret_cast<const uint4*>(&tile[(sub * 16 + col) * ROW + j0]);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, raw), qb[c],
                                                     acc, 0, 0, 0);
      }
      // D layout: this lane holds points sub*16 + 4*grp + i of window col
      uint32_t keys[4];
      int nk = 0;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int r = sub * 16 + 4 * grp + i;
        const int64_t p = t0 + r;
        const float ap = tnorm[r] + qn - 2.0f * acc[i];
        const uint32_t key = win_key(ap, (uint32_t)(p - ws));
        const bool take = wvalid && p >= ws && p <= we && key < tau;
        keys[i] = key;
        nk += take ? 1 : 0;
        if (!take) keys[i] = 0xFFFFFFFFu;
      }
      if (nk > 0) {
        int at = atomicAdd(mycnt, nk);
#pragma unroll
        for (int i = 0; i < 4; i++)
          if (keys[i] != 0xFFFFFFFFu) mybuf[at++] = keys[i];
      }
    }
    __syncthreads();                           // buffer counts complete, tile reusable
    // windows whose buffer could overflow during the next tile are merged now
    const uint32_t need =
        (uint32_t)ballot(lane < kScanWinPerWave && cnt[wave][lane] > BUF - TP) & 0xFFFFu;
    if (need) flush(need);
  }
  const uint32_t rest = (uint32_t)ballot(lane < kScanWinPerWave && cnt[wave][lane] > 0) & 0xFFFFu;
  if (rest) flush(rest);
  // write each valid window's list (64E 32-bit keys)
#pragma unroll
  for (int w = 0; w < kScanWinPerWave; w++) {
    const int64_t wj = wbase + wave * kScanWinPerWave + w;
    if (wj < nw) {
      const int32_t id = S.win_order ? S.win_order[wj] : (int32_t)wj;
      uint32_t* out = reinterpret_cast<uint32_t*>(S.cand + (int64_t)id * S.cand_stride);
#pragma unroll
      for (int e = 0; e < E; e++) out[e * kWave + lane] = L[w][e];
    }
  }
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
    const uint32_t* c = reinterpret_cast<const uint32_t*>(S.cand + (int64_t)(w0 + j) * S.cand_stride);
    const int64_t wsj = S.win_s[w0 + j];
    uint64_t B[E];
#pragma unroll
    for (int e = 0; e < E; e++) B[e] = cand_key(c[e * kWave + lane], wsj);
    if (j == 0) {
#pragma unroll
      for (int e = 0; e < E; e++) L[e] = B[e];
    } else {
      list_merge(L, B, cap, lane);
    }
  }
  // float32 rerank of the first mr candidates
  const int mr = S.mr;
  const float* q = S.queries + (int64_t)qi * S.dq;
  float qr32[CPL32][4];
  load_query<kF32, G32, CPL32>(q, S.dq, lane, qr32);
  SearchArgs A;
  A.vec = S.vec;
  A.d = S.d;
  A.dq = S.dq;
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
      key = sort32(key, lane, n_new);
      merge_sorted32(R, key, k, lane);
    }
  }
  // certification
  const uint64_t kth = list_at(R, k - 1);
  const uint64_t next = mr < cap ? list_at(L, mr) : kKeyInf;  // (mr+1)-th key: a lower bound
  bool certified = true;
  if (next != kKeyInf && kth != kKeyInf) {
    // |approx - exact| <= 2 (dx + dq + dx dq) |x||q|            (bfloat16 rounding)
    //                    + gamma (2 |x||q| (1+dx)(1+dq) + |x|^2 + |q|^2)  (float32 sums)
    float qn = 0.0f, dq = 0.0f;
    for (int j = lane; j < S.dq; j += kWave) {
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
  A.dq = S.dq;
  A.dp = S.dp;
  for (int64_t t = 0; t < nfb; t++) {
    const int32_t qi = S.fb_list[t];
    const int64_t w0 = S.q_win0[qi], nwq = S.q_nwin[qi];
    if (gw >= nwq) continue;
    float qr32[CPL32][4];
    load_query<kF32, G32, CPL32>(S.queries + (int64_t)qi * S.dq, S.dq, lane, qr32);
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
