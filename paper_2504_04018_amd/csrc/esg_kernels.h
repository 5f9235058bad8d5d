// Argument block shared by the search kernels and the host runtime.
#pragma once

#include <stdint.h>

#include "../../include/esg.h"

namespace esgk {

constexpr int kWavesPerGroup = 4;   // independent waves per workgroup
constexpr int kBatch = 32;          // adjacency slots handled per expansion (max degree)
constexpr int kStageBytes = 1024;   // per-wave LDS staging ahead of the hash

enum DistKind : int { kF32 = 0, kBF16 = 1, kFP8 = 2 };

struct SearchArgs {
  // index (device)
  const float* vec;       // [n][dp] float32, rows zero-padded to dp
  const uint16_t* vec16;  // [n][dp] bfloat16 bits or null
  const uint8_t* vec8;    // [n][dp] fp8 e4m3 codes or null
  const float* scale8;    // [n] fp8 scales or null
  const uint32_t* adj;    // [n_depth][n][R]
  const uint32_t* ep;     // [2^n_depth]
  const int64_t* ext_id;  // [n]
  int64_t n;
  int32_t d, dp, R, leaf, n_depth, c_den;
  // batch
  const float* queries;   // [nq][d]
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
  uint32_t* spill;        // [slots][spill_words] visited bitmaps used after the LDS hash fills
  int64_t spill_words;
  int64_t spill_slots;
  uint32_t* counter;      // work-queue head
  const int32_t* qlist;   // queries to process (null = 0..nq-1)
  const int32_t* qcount;  // device count of qlist (null = nq)
  int32_t hash_cap;       // 16-bit LDS visited slots per wave (power of two)
  int32_t pad_;
};

}  // namespace esgk
