// Table of compiled search kernels for one vector dimension.
#pragma once

namespace esgk {

constexpr int kNumKinds = 3;    // float32, bfloat16, fp8 traversal
constexpr int kNumWidths = 5;   // list words per lane E = 1, 2, 4, 8, 16

constexpr int kNumScanWidths = 3;  // scan candidate lists of 64, 128, 256 keys

struct KernelTable {
  int dim;
  const void* fn[kNumKinds][kNumWidths][3];   // [.][.][0] plain, [1] one-hop probe, [2] longer probe
  const void* scan_select[kNumScanWidths];  // MFMA distances + per-window top list
  const void* rerank[kNumScanWidths];     // merge + float32 rerank + certificate
  const void* fallback[kNumScanWidths];   // exact float32 scan of each window
  const void* fb_merge[kNumScanWidths];   // merge of the windows' exact lists
  const void* build_search[kNumWidths];   // builder: float32 insertion searches
  const void* build_prune;                // builder: forward rows by occlusion
  const void* build_reverse;              // builder: reverse edges
};

}  // namespace esgk
