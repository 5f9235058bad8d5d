// The persistent search kernel (see esg_search_impl.h for the data layout).
#pragma once

#include "esg_search_impl.h"

namespace esgk {

constexpr int kInsertMax = 4;   // batches with at most this many survivors are inserted one by one

struct PartStats {
  int64_t hops;
  int64_t n_visited;
};

// Alg. 1 with POST on graph node [a,b] of tree depth `depth`; results (the
// final Q, at most m keys) are left in Q.
// Features of a graph part after the probe (all wave-uniform scalars).
struct ProbeCtx {
  int64_t w_query;   // width of the whole query range
  int n_parts;
  float* feat;       // where to write the features (or null)
};

// 12 -> 64 -> 64 -> 1 ReLU network, one hidden unit per lane.  Weights in
// the packed layout: W1 and W2 as [input/4][hidden unit][4], so each lane
// reads its unit's weights 16 bytes at a time and a wave's read is one
// contiguous kilobyte.  Loads go in rounds of kMlpRound float4 per lane;
// each round's addresses depend on the previous round's sum, so the
// compiler cannot issue them all at once: the network then adds few
// registers on top of the live search state.  Lane i < 12 holds feature i
// in `f`; returns the raw output on every lane.  The normalised inputs and
// the first hidden layer pass through the wave's LDS staging.
constexpr int kMlpRound = 2;

__device__ __forceinline__ float mlp_infer(const float* __restrict__ P, float f, WaveLds* Ls,
                                           int lane) {
  const float4* __restrict__ w1 = reinterpret_cast<const float4*>(P + kOffW1);
  const float4* __restrict__ w2 = reinterpret_cast<const float4*>(P + kOffW2);
  Ls->fstage[lane] = lane < kFeat ? (f - P[kOffMu + lane]) / P[kOffSd + lane] : 0.0f;
  wave_lds_sync();
  const float4* xs = reinterpret_cast<const float4*>(Ls->fstage);
  auto layer = [&](const float4* __restrict__ w, int n4, float acc) {
    for (int r = 0; r < n4; r += kMlpRound) {
      int col = lane;
      asm volatile("" : "+v"(col) : "v"(acc));
      float4 b[kMlpRound];
#pragma unroll
      for (int c = 0; c < kMlpRound; c++) b[c] = w[(r + c) * kHidden + col];
#pragma unroll
      for (int c = 0; c < kMlpRound; c++) {
        const float4 x = xs[r + c];
        acc = __builtin_fmaf(b[c].x, x.x, acc);
        acc = __builtin_fmaf(b[c].y, x.y, acc);
        acc = __builtin_fmaf(b[c].z, x.z, acc);
        acc = __builtin_fmaf(b[c].w, x.w, acc);
      }
    }
    return acc > 0.0f ? acc : 0.0f;
  };
  static_assert(kFeat % 4 == 0 && (kFeat / 4) % 1 == 0, "feature count");
  float h1 = 0.0f;
  {
    // W1: kFeat/4 = 3 float4 per lane, one at a time
    float acc = P[kOffB1 + lane];
    for (int c = 0; c < kFeat / 4; c++) {
      int col = lane;
      asm volatile("" : "+v"(col) : "v"(acc));
      const float4 b = w1[c * kHidden + col];
      const float4 x = xs[c];
      acc = __builtin_fmaf(b.x, x.x, acc);
      acc = __builtin_fmaf(b.y, x.y, acc);
      acc = __builtin_fmaf(b.z, x.z, acc);
      acc = __builtin_fmaf(b.w, x.w, acc);
    }
    h1 = acc > 0.0f ? acc : 0.0f;
  }
  wave_lds_sync();
  Ls->fstage[lane] = h1;
  wave_lds_sync();
  const float h2 = layer(w2, kHidden / 4, P[kOffB2 + lane]);
  float y = P[kOffW3 + lane] * h2;
#pragma unroll
  for (int s = 1; s < kWave; s <<= 1) y = y + xor_f(y, s, lane);
  wave_lds_sync();
  return y + P[kOffB3];
}

// Feature `lane` (lanes 0..11) of a graph part after the probe, from the
// wave-uniform state: log2 of the part's filter width and node size, their
// ratio, log2 of the query width, number of parts - 1, fill of P's live part
// and of Q
// (relative to k, at most 4), in-range share of the visited points, the
// best and k-th distances in Q and the best distance in P relative to the
// entry's (or to the k-th), log2(1 + visited).
__device__ __forceinline__ float probe_feature(int lane, float wp, float L, int64_t w_query,
                                               int n_parts, int psize, int cap_p, int qsize,
                                               int k, int64_t n_inr, int64_t nvis, float q0,
                                               float qk, float p0, float den) {
  const float lg_arg = lane == 0 ? wp : lane == 1 ? L : lane == 3 ? (float)w_query
                                   : 1.0f + (float)nvis;
  const float lg = __log2f(lg_arg);
  float num = 1.0f, dv = 1.0f;
  switch (lane) {
    case 2: num = wp; dv = L; break;
    case 5: num = (float)psize; dv = (float)cap_p; break;
    case 6: num = (float)qsize; dv = (float)k; break;
    case 7: num = (float)n_inr; dv = (float)nvis; break;
    case 8: num = q0; dv = den; break;
    case 9: num = qk; dv = den; break;
    case 10: num = qk > 0.0f ? p0 : 1.0f; dv = qk > 0.0f ? qk : 1.0f; break;
    default: break;
  }
  float f = num / dv;
  if (lane == 6) f = fminf(f, 4.0f);
  if (lane == 0 || lane == 1 || lane == 3 || lane == 11) f = lg;
  if (lane == 4) f = (float)(n_parts - 1);
  return f;
}

// Gather rounds in flight per lane: 8 in every kernel.
template <int KIND, int LEARN>
constexpr int kLearnRF = 8;
// Rounds reduced together (reduce-scatter) in the distance pass: all of them
// for float32; the narrow-storage kernels reduce one round at a time
// (measured faster there: fewer registers, also in the learned kernels).
template <int KIND, int LEARN>
constexpr int kReduceGroup = KIND == kF32 ? 8 : 1;

template <int KIND, int G, int CPL, int E, int LEARN>
__device__ __forceinline__ PartStats search_graph(const SearchArgs& A, WaveLds* Ls, Visited& V,
                                                  const Part& pt, int m, int cap_p,
                                                  const float (&qr)[CPL][Traits<KIND>::W],
                                                  uint64_t (&Q)[E], uint32_t* dump, int lane,
                                                  const ProbeCtx& pc) {
  uint64_t P[E];
  list_clear(P);
  list_clear(Q);
  visited_reset(A, V, pt.a, pt.b, lane);
  const uint32_t* rows = A.adj + A.row_base[pt.depth] * (int64_t)A.R;
  const uint32_t ep = A.ep[pt.heap];

  // The entry's adjacency row is requested together with its vector, so the
  // two loads overlap.
  uint32_t vrow = lane < A.R ? rows[(size_t)ep * A.R + lane] : kNoNode;

  // P <- ep ; Q <- ep when ep is in range (POST)
  visit(A, V, ep, lane == 0, lane);
  float dep = batch_dist<KIND, G, CPL>(A, ep, 1, qr, Ls, lane);
  const uint64_t kep = make_key(__uint_as_float(readlane(__float_as_uint(dep), 0)), ep);
  if (lane == 0) {
    P[0] = kep;
    if (ep >= pt.x && ep <= pt.y) Q[0] = kep;
  }
  if (dump && lane == 0 && A.visited_cap > 0) dump[0] = ep;
  // 32-bit counters (a part visits at most its n < 2^32 positions) keep
  // the scalar registers of the hop loop few
  uint32_t nvis = 1, hops = 0;
  uint32_t n_inr = (ep >= pt.x && ep <= pt.y) ? 1 : 0;  // visited points inside [x,y]
  const float d_ep = key_dist(kep);
  // expansions allowed (hop_budget < 0: unbounded, kept as 2^32 - 1)
  uint32_t hop_limit = (A.hop_budget < 0 || A.hop_budget > 0xFFFFFFFFll)
                           ? 0xFFFFFFFFu : (uint32_t)A.hop_budget;

  // The row of the next candidate is fetched as soon as that candidate is
  // known (right after the new batch is sorted), so the load overlaps the
  // merges of the current expansion.
  uint64_t u = kep;                                          // P[0]; its row is vrow
  // One expansion of Alg. 1 (pop the nearest candidate, visit its
  // neighbours, score the new ones, merge them into P and Q); false when the
  // search (or, in the probe phase, the probe) ends instead.
  auto hop = [&](bool probe_phase) -> bool {
    {
      if (u == kKeyInf) return false;                            // P is empty
      if (probe_phase && hops == (uint32_t)A.probe_hops) return false;  // probe over: switch first
      const uint64_t worst = list_at(Q, m - 1);
      if (worst != kKeyInf && worst < u) return false;           // farther than a full Q
      if (hops >= hop_limit) return false;
      list_pop(P, lane);
      hops++;

      const uint32_t v = vrow;
      const bool is_new = visit(A, V, v, v != kNoNode && v >= pt.a && v <= pt.b, lane);
      const uint64_t nm = ballot(is_new);
      const int n_new = __popcll(nm);
      if (n_new == 0) {
        u = readlane64(P[0], 0);
        vrow = (lane < A.R && u != kKeyInf) ? rows[(size_t)key_pos(u) * A.R + lane] : kNoNode;
        return true;
      }
      // the new ids to lanes 0..n_new-1 in lane order (the others fill the
      // remaining lanes, so the push is a permutation)
      const int rn = rank_below(nm);
      const uint32_t pushed = push(v, is_new ? rn : n_new + (lane - rn));
      const uint32_t nid = lane < n_new ? pushed : kNoNode;
      if (__builtin_expect(dump != nullptr, 0)) {   // a uniform branch: the test is not folded
        if (lane < n_new && (int64_t)nvis + lane < A.visited_cap) dump[nvis + lane] = nid;
      }
      nvis += n_new;
      if (probe_phase) n_inr += __popcll(ballot(lane < n_new && nid >= pt.x && nid <= pt.y));

      constexpr int kRF = kLearnRF<KIND, LEARN>, kTG = kReduceGroup<KIND, LEARN>;
      const float bd = batch_dist<KIND, G, CPL, kRF, kTG>(A, nid, n_new, qr, Ls, lane);
      uint64_t key = lane < n_new ? make_key(bd, nid) : kKeyInf;
      // A key that loses to a full Q can neither enter Q nor ever be expanded
      // (the bound only tightens), so dropping it leaves P's useful part, Q
      // and every later step unchanged.
      if (worst != kKeyInf && worst < key) key = kKeyInf;
      const uint64_t sm = ballot(key != kKeyInf);
      const uint64_t p0 = readlane64(P[0], 0);
      if (sm == 0) {
        u = p0;
        vrow = (lane < A.R && u != kKeyInf) ? rows[(size_t)key_pos(u) * A.R + lane] : kNoNode;
        return true;
      }
      if (__popcll(sm) <= kInsertMax) {
        // few survivors: insert them one by one
        uint64_t bmin = kKeyInf;
        for (uint64_t mm = sm; mm; mm &= mm - 1) bmin = kmin(bmin, readlane64(key, __builtin_ctzll(mm)));
        u = kmin(p0, bmin);
        vrow = (lane < A.R && u != kKeyInf) ? rows[(size_t)key_pos(u) * A.R + lane] : kNoNode;
        for (uint64_t mm = sm; mm; mm &= mm - 1) {
          const uint64_t kj = readlane64(key, __builtin_ctzll(mm));
          list_insert(P, kj, cap_p, lane);
          const uint32_t pj = key_pos(kj);
          if (pj >= pt.x && pj <= pt.y) list_insert(Q, kj, m, lane);
        }
        return true;
      }
      key = sort32(key, lane, n_new);
      const uint64_t kmin0 = readlane64(key, 0);
      u = kmin(p0, kmin0);                                       // min of P after the merge
      vrow = (lane < A.R && u != kKeyInf) ? rows[(size_t)key_pos(u) * A.R + lane] : kNoNode;
      merge_sorted32(P, key, cap_p, lane);
      const uint32_t kp = key_pos(key);
      const bool inr = lane_in(0xFFFFFFFFull) && key != kKeyInf && kp >= pt.x && kp <= pt.y;
      const uint64_t qm = ballot(inr);
      if (qm != 0) {
        // the in-range keys, reversed into lanes 31, 30, ... (a list of at
        // most 32) or 63, 62, ...
        // (one permutation: the other lanes fill lanes 0..top-nq and
        // top+1..63 with +inf)
        const bool low = E == 1 && m <= 32;
        const int top = low ? 31 : 63, nq = __popcll(qm), rq = rank_below(qm);
        const int ro = lane - rq;
        const int dst = inr ? top - rq : (ro <= top - nq ? ro : ro + nq);
        const uint64_t rev = push64(inr ? key : kKeyInf, dst);
        if (low)
          merge_low32(Q[0], rev, m, lane);
        else
          list_merge32(Q, rev, m, lane);
      }
    }
    return true;
  };
  // Plain kernel: hops until the search ends.  Learned kernel with a one-hop
  // probe: the first hop and the switch come before the loop, which is then
  // the plain kernel's loop.  Learned kernel with a longer probe: a probe
  // loop, the switch, then the main loop.
  bool go = true;
  if constexpr (LEARN == 1) {
    go = A.probe_hops == 1 && hop(true);
  } else if constexpr (LEARN == 2) {
    while (hop(true)) {
    }
  }
  // The switch is taken only when the search goes on past the probe (its
  // next candidate passes the stop test); P's fill counts its live part
  // (candidates not farther than a full Q's worst), which the lossless
  // prune leaves unchanged.
  constexpr bool kLearned = LEARN == 1 || LEARN == 2;
  const uint64_t worst0 = (kLearned && go) ? list_at(Q, m - 1) : kKeyInf;
  if (kLearned && go && u != kKeyInf && hops == (uint32_t)A.probe_hops && !(worst0 < u)) {
    // probe over: features -> predicted beam width or stopping step
    int qsize = 0, psize = 0;
#pragma unroll
    for (int e = 0; e < E; e++) {
      qsize += __popcll(ballot(Q[e] != kKeyInf));
      psize += __popcll(ballot(P[e] != kKeyInf && P[e] <= worst0));
    }
    const int kk = A.k < qsize ? A.k : qsize;
    const float q0 = qsize > 0 ? key_dist(list_at(Q, 0)) : d_ep;
    const float qk = kk > 0 ? key_dist(list_at(Q, kk - 1)) : d_ep;
    const float f = probe_feature(lane, (float)(pt.y - pt.x + 1), (float)(pt.b - pt.a + 1),
                                  pc.w_query, pc.n_parts, psize, cap_p, qsize, A.k, n_inr,
                                  nvis, q0, qk, key_dist(u), d_ep > 0.0f ? d_ep : 1.0f);
    float y = 0.0f;
    int efp = m;
    if (A.mlp) {
      y = mlp_infer(A.mlp, f, Ls, lane);
      const float e2 = exp2f(y + A.mlp_delta);
      if (A.mlp_target == 1) {
        // stopping step: the part may take ceil(2^(y + delta)) more expansions
        const int64_t more = e2 >= 1.0e9f ? (int64_t)1000000000
                                          : (int64_t)ceilf(e2 < 1.0f ? 1.0f : e2);
        if ((int64_t)hops + more < (int64_t)hop_limit) hop_limit = (uint32_t)(hops + more);
        efp = (int)more;
      } else {
        efp = e2 >= (float)m ? m : (int)ceilf(e2);
        efp = efp < A.k ? A.k : efp;
        // continue with m = cand_cap = ef': keep the ef' best of P and Q
#pragma unroll
        for (int e = 0; e < E; e++)
          if (e * kWave + lane >= efp) {
            P[e] = kKeyInf;
            Q[e] = kKeyInf;
          }
        m = efp;
        cap_p = efp;
        u = readlane64(P[0], 0);
      }
    }
    if (pc.feat) {
      if (lane < kFeat) pc.feat[lane] = f;
      if (lane == 0) {
        pc.feat[kFeat] = y;
        pc.feat[kFeat + 1] = (float)efp;
      }
    }
  }
  if (go)
    while (hop(false)) {
    }
  visited_finish(A, V, lane);
  return {hops, nvis};
}

// Scores positions [x,y] (a leaf) with float32 distances; keeps the best k.
template <int G32, int CPL32, int E>
__device__ __forceinline__ void scan_leaf(const SearchArgs& A, WaveLds* Ls, const Part& pt, int k,
                                          const float (&qr32)[CPL32][4], uint64_t (&R)[E],
                                          int lane) {
  list_clear(R);
  for (uint32_t base = pt.x; base <= pt.y; base += kBatch) {
    const int n_new = (int)((pt.y - base + 1) < (uint32_t)kBatch ? (pt.y - base + 1) : kBatch);
    const uint32_t nid = lane < n_new ? base + (uint32_t)lane : kNoNode;
    const float bd = batch_dist<kF32, G32, CPL32>(A, nid, n_new, qr32, Ls, lane);
    uint64_t key = lane < n_new ? make_key(bd, nid) : kKeyInf;
    const uint64_t worst = list_at(R, k - 1);
    if (worst != kKeyInf && worst < key) key = kKeyInf;
    const uint64_t sm = ballot(key != kKeyInf);
    if (sm != 0 && __popcll(sm) <= kInsertMax) {
      for (uint64_t mm = sm; mm; mm &= mm - 1)
        list_insert(R, readlane64(key, __builtin_ctzll(mm)), k, lane);
    } else if (sm != 0) {
      key = sort32(key, lane, n_new);
      merge_sorted32(R, key, k, lane);
    }
    if (base > 0xFFFFFFFFu - kBatch) break;
  }
}

// Recomputes every key of Q with float32 distances and keeps the best k.
template <int G32, int CPL32, int E>
__device__ __forceinline__ void rerank_f32(const SearchArgs& A, WaveLds* Ls, int k,
                                           const float (&qr32)[CPL32][4], uint64_t (&Q)[E],
                                           int lane) {
  uint64_t R[E];
  list_clear(R);
#pragma unroll
  for (int e = 0; e < E; e++) {
#pragma unroll
    for (int s = 0; s < kWave / kBatch; s++) {
      const uint64_t kq = bperm64(Q[e], (s * kBatch + lane) & 63);  // lanes < 32: block s
      const bool ok = lane < kBatch && kq != kKeyInf;
      const int n_new = __popcll(ballot(ok));
      if (n_new == 0) continue;
      const uint32_t nid = ok ? key_pos(kq) : kNoNode;
      const float bd = batch_dist<kF32, G32, CPL32>(A, nid, n_new, qr32, Ls, lane);
      uint64_t key = lane < n_new ? make_key(bd, nid) : kKeyInf;
      key = sort32(key, lane, n_new);
      merge_sorted32(R, key, k, lane);
    }
  }
#pragma unroll
  for (int e = 0; e < E; e++) Q[e] = R[e];
}

template <int KIND, int G, int CPL, int G32, int CPL32, int E, int LEARN>
__device__ __forceinline__ void process_query(const SearchArgs& A, WaveLds* Ls, Visited& V,
                                              int64_t qi, int lane) {
  const int k = A.k;
  int64_t* ids = A.ids + qi * k;
  float* dists = A.dists + qi * k;
  const int64_t lq = A.l[qi], rq = A.r[qi];
  const bool valid = lq >= 0 && rq < A.n && lq <= rq;
  Part pt{};
  int np = 0;
  if constexpr (LEARN == kBuildSearch) {
    // the builder's insertion search: the graph of one depth on [l, r]
    if (valid) pt = Part{1, A.forced_depth, qi, (uint32_t)lq, (uint32_t)rq, (uint32_t)lq, (uint32_t)rq};
    np = valid ? 1 : 0;
  } else {
    np = valid ? select_parts(A, lq, rq, 0, pt) : 0;
  }
  if (!valid || np < 0) {
    for (int i = lane; i < k; i += kWave) {
      ids[i] = -1;
      dists[i] = __int_as_float(0x7F800000);
    }
    if (lane == 0 && A.n_invalid) atomicAdd((unsigned long long*)A.n_invalid, 1ull);
    if (A.trace && lane < 2) A.trace[qi * 2 + lane].kind = 0;
    return;
  }

  const float* q = A.queries + qi * (int64_t)A.dq;
  float qr[CPL][Traits<KIND>::W];
  load_query<KIND, G, CPL>(q, A.dq, lane, qr);

  const int m = A.ef;
  const int cap_p = A.cand_cap;
  uint64_t Res[E];
  list_clear(Res);
  // One copy of the part code (not unrolled: half the instruction footprint).
#pragma nounroll
  for (int p = 0; p < np; p++) {
    if (p == 1) select_parts(A, lq, rq, 1, pt);
    uint64_t Qp[E];
    PartStats st{0, 0};
    const uint64_t t_start = A.trace ? __builtin_amdgcn_s_memrealtime() : 0;
    if (pt.kind == 2) {
      if constexpr (KIND == kF32) scan_leaf<G, CPL, E>(A, Ls, pt, k, qr, Qp, lane);
      else {
        float qr32[CPL32][4];               // loaded where needed, not kept across the search
        load_query<kF32, G32, CPL32>(q, A.dq, lane, qr32);
        scan_leaf<G32, CPL32, E>(A, Ls, pt, k, qr32, Qp, lane);
      }
      st.n_visited = (int64_t)(pt.y - pt.x) + 1;
    } else {
      uint32_t* dump = A.visited ? A.visited + (qi * 2 + p) * A.visited_cap : nullptr;
      ProbeCtx pc;
      pc.w_query = rq - lq + 1;
      pc.n_parts = np;
      pc.feat = A.feat_out ? A.feat_out + (qi * 2 + p) * kFeatStride : nullptr;
      // a beam chosen per part before the search (m = cand_cap = ef')
      const int pe = A.part_ef ? A.part_ef[qi * 2 + p] : m;
      const int mp = pe < A.k ? A.k : (pe > m ? m : pe);
      const int cp = A.part_ef ? mp : cap_p;
      st = search_graph<KIND, G, CPL, E, LEARN>(A, Ls, V, pt, mp, cp, qr, Qp, dump, lane, pc);
      if constexpr (KIND != kF32)
        if (A.rerank) {
          float qr32[CPL32][4];
          load_query<kF32, G32, CPL32>(q, A.dq, lane, qr32);
          rerank_f32<G32, CPL32, E>(A, Ls, k, qr32, Qp, lane);
        }
#pragma unroll
      for (int e = 0; e < E; e++)
        if (e * kWave + lane >= k) Qp[e] = kKeyInf;
    }
    list_merge(Res, Qp, k, lane);
    if (A.trace && lane == 0) {
      esg_part_trace& tr = A.trace[qi * 2 + p];
      tr.kind = pt.kind;
      tr.depth = pt.depth;
      tr.heap = pt.heap;
      tr.a = pt.a;
      tr.b = pt.b;
      tr.x = pt.x;
      tr.y = pt.y;
      tr.hops = st.hops;
      tr.n_visited = st.n_visited;
      tr.ticks = (int64_t)(__builtin_amdgcn_s_memrealtime() - t_start);
    }
  }
  if (A.trace && lane == 0 && np < 2) A.trace[qi * 2 + 1].kind = 0;
#pragma unroll
  for (int e = 0; e < E; e++) {
    const int i = e * kWave + lane;
    if (i < k) {
      const uint64_t key = Res[e];
      ids[i] = key == kKeyInf ? -1 : A.ext_id[key_pos(key)];
      dists[i] = key == kKeyInf ? __int_as_float(0x7F800000) : key_dist(key);
    }
  }
}

// Occupancy target: the float32 kernels with lists of up to 128 keys and the
// bfloat16 kernels with 64 keys are held to 4 waves per SIMD (measured: the
// few spills this costs are cheaper than a lost wave on these latency-bound
// kernels), except the bfloat16 kernel with the one-hop probe, whose
// predictor sits before the loop and spills into it at 4 (3 waves measured
// 15 % faster); the others keep the compiler's choice.
template <int KIND, int E, int LEARN>
constexpr int min_waves() {
  if (KIND == kBF16 && E == 1 && LEARN == 1) return 3;
  return ((KIND == kF32 && E <= 2) || (KIND == kBF16 && E == 1)) ? 4 : 1;
}

template <int KIND, int G, int CPL, int G32, int CPL32, int E, int LEARN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(min_waves<KIND, E, LEARN>(), 8)))
void search_kernel(SearchArgs A) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int lane = lane_id();
  const int wid = (int)(threadIdx.x >> 6);
  WaveLds* Ls = reinterpret_cast<WaveLds*>(smem + (size_t)wid * (kStageBytes + 2 * A.hash_cap));
  const int64_t slot = (int64_t)blockIdx.x * kWavesPerGroup + wid;
  Visited V;
  V.table = wave_table(Ls);
  V.bm = A.spill + slot * (A.spill_words + kSpillLog);
  V.a = V.b = 0;
  V.kb = V.shift = 0;
  V.kb_mask = 0;
  V.nlog = 0;
  const int64_t count = A.qcount ? (int64_t)*A.qcount : A.nq;
  for (;;) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(A.counter, 1u);
    const int64_t ti = (int64_t)readlane(t, 0);
    if (ti >= count) break;
    const int64_t qi = A.qlist ? (int64_t)A.qlist[ti] : ti;
    process_query<KIND, G, CPL, G32, CPL32, E, LEARN>(A, Ls, V, qi, lane);
  }
}

}  // namespace esgk
