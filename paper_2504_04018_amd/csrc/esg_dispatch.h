// Table of compiled search kernels for one vector dimension.
#pragma once

namespace esgk {

constexpr int kNumKinds = 3;    // float32, bfloat16, fp8 traversal
constexpr int kNumWidths = 5;   // list words per lane E = 1, 2, 4, 8, 16

struct KernelTable {
  int dim;
  const void* fn[kNumKinds][kNumWidths];
};

}  // namespace esgk
