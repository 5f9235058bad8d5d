// Argument block shared by the search kernels and the host runtime.
#pragma once

#include <stdint.h>

#include "../../include/esg.h"

namespace esgk {

constexpr int kWavesPerGroup = 4;   // independent waves per workgroup
constexpr int kBatch = 32;          // adjacency slots handled per expansion (max degree)
constexpr int kStageBytes = 1024;   // per-wave LDS staging ahead of the hash

enum DistKind : int { kF32 = 0, kBF16 = 1, kFP8 = 2 };
// Search kernel variants (template argument LEARN): 0 plain, 1 learned
// switch after a one-hop probe, 2 after a longer probe, kBuildSearch the
// builder's insertion search (plain, with the part given per query).
constexpr int kBuildSearch = 3;

// Beam-width predictor: 12 features -> 64 -> 64 -> 1 (ReLU), float32.
// Parameter layout: W1[64][12] b1[64] W2[64][64] b2[64] W3[64] b3[1]
// feature mean[12] feature scale[12].
constexpr int kFeat = 12;
constexpr int kHidden = 64;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHidden * kFeat;
constexpr int kOffW2 = kOffB1 + kHidden;
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;
constexpr int kOffW3 = kOffB2 + kHidden;
constexpr int kOffB3 = kOffW3 + kHidden;
constexpr int kOffMu = kOffB3 + 1;
constexpr int kOffSd = kOffMu + kFeat;
constexpr int kMlpParams = kOffSd + kFeat;   // 5081
constexpr int kMlpWeights = kOffMu;           // 5057 trainable
constexpr int kFeatStride = 16;               // 12 features, raw output, ef', 2 spare

struct SearchArgs {
  // index (device)
  const float* vec;       // [n][dp] float32, rows zero-padded to dp
  const uint16_t* vec16;  // [n][dp] bfloat16 bits or null
  const uint8_t* vec8;    // [n][dp] fp8 e4m3 codes or null
  const float* scale8;    // [n] fp8 scales or null
  const uint32_t* adj;    // rows of every depth, addressed through row_base
  const uint32_t* ep;     // [2^n_depth]
  const int64_t* ext_id;  // [n]
  int64_t n;
  int32_t d, dp, R, leaf, n_depth, c_den;
  int32_t dq;             // values per query row (<= d; the rest of a query reads as 0)
  int32_t fanout;         // children per tree node (the chains' base in layout 1)
  int32_t layout;         // 0: segment tree; 1: prefix and suffix chains (half-bounded index)
  const int64_t* row_base;// [n_depth]: row of position p at depth t is adj + (row_base[t] + p) R
  // builder's insertion searches (the kBuildSearch kernels): query i
  // searches the graph of depth forced_depth on [l[i], r[i]] from ep[i]
  int32_t forced_depth;
  // batch
  const float* queries;   // [nq][dq]
  const int64_t* l;
  const int64_t* r;
  int64_t nq;
  int32_t k, ef, cand_cap, rerank;
  int64_t hop_budget;
  int64_t* ids;
  float* dists;
  // optional debug output
  esg_part_trace* trace;
  uint32_t* visited;
  int64_t visited_cap;
  int64_t* n_invalid;
  // workspace
  uint32_t* spill;        // [slots][spill_words + spill log] visited bitmaps (all zero
                          // between parts) used after the LDS hash fills, and their logs
  int64_t spill_words;
  int64_t spill_slots;
  uint32_t* counter;      // work-queue head
  // learned beam width: after probe_hops expansions at m = ef the MLP sets
  // m = cand_cap = ef' for the rest of the part
  const float* mlp;       // packed parameters (kMlpParams floats: W1, W2 input-major) or null
  float* feat_out;        // [nq][2][kFeatStride] features, raw output and ef' (optional)
  int32_t probe_hops;
  const int32_t* part_ef; // [nq][2] beam of each graph part chosen before the search, or null
  float mlp_delta;        // calibration offset added to the predicted log2 value
  int32_t mlp_target;     // 0: the output sets the beam width, 1: the remaining hops
  const int32_t* qlist;   // queries to process (null = 0..nq-1)
  const int32_t* qcount;  // device count of qlist (null = nq)
  int32_t hash_cap;       // 16-bit LDS visited slots per wave (power of two)
  int32_t pad_;
};

}  // namespace esgk
