// Instantiates the search kernels for one vector dimension (-DESG_DIM=d).
#include "esg_build_impl.h"
#include "esg_dispatch.h"
#include "esg_scan_impl.h"

#ifndef ESG_DIM
#error "compile with -DESG_DIM=<dimension>"
#endif

namespace esgk {
namespace {

constexpr int lanes_for(int chunks) {
  int g = 1;
  while (g < chunks) g *= 2;
  return g > 64 ? 64 : g;
}

template <int KIND>
struct Shape {
  static constexpr int C = (ESG_DIM + Traits<KIND>::W - 1) / Traits<KIND>::W;
  static constexpr int G = lanes_for(C);
  static constexpr int CPL = (C + G - 1) / G;
};

template <int KIND, int E, int LEARN>
const void* kernel_ptr() {
  using S = Shape<KIND>;
  using S32 = Shape<kF32>;
  return reinterpret_cast<const void*>(
      &search_kernel<KIND, S::G, S::CPL, S32::G, S32::CPL, E, LEARN>);
}

template <int KIND, int LEARN>
void fill_one(KernelTable* t) {
  t->fn[KIND][0][LEARN] = kernel_ptr<KIND, 1, LEARN>();
  t->fn[KIND][1][LEARN] = kernel_ptr<KIND, 2, LEARN>();
  t->fn[KIND][2][LEARN] = kernel_ptr<KIND, 4, LEARN>();
  t->fn[KIND][3][LEARN] = kernel_ptr<KIND, 8, LEARN>();
  t->fn[KIND][4][LEARN] = kernel_ptr<KIND, 16, LEARN>();
}

template <int KIND>
void fill(KernelTable* t) {
  fill_one<KIND, 0>(t);   // plain
  fill_one<KIND, 1>(t);   // learned switch after a one-hop probe
  fill_one<KIND, 2>(t);   // learned switch after a longer probe
}

constexpr int kDp = (ESG_DIM + 15) / 16 * 16;
constexpr int kNK = (kDp + 31) / 32;
// positions per LDS tile of the scan: the staged tile stays within 32 KB
constexpr int kTP = kDp <= 128 ? 64 : (kDp <= 256 ? 32 : 16);
// the scan stages a tile of kTP rows in LDS: compiled up to rows of 1,024
constexpr bool kHasScan = kDp <= 1024;

template <int E>
void fill_scan(KernelTable* t, int slot) {
  using S32 = Shape<kF32>;
  if constexpr (kHasScan)
    t->scan_select[slot] = reinterpret_cast<const void*>(&scan_select_kernel<kNK, E, kTP, kDp>);
  t->rerank[slot] = reinterpret_cast<const void*>(&rerank_kernel<S32::G, S32::CPL, E>);
  t->fallback[slot] = reinterpret_cast<const void*>(&fallback_window_kernel<S32::G, S32::CPL, E>);
  t->fb_merge[slot] = reinterpret_cast<const void*>(&fallback_merge_kernel<E>);
}

}  // namespace
}  // namespace esgk

#define ESG_CAT2(a, b) a##b
#define ESG_CAT(a, b) ESG_CAT2(a, b)

extern "C" void ESG_CAT(esg_register_dim_, ESG_DIM)(esgk::KernelTable* t) {
  t->dim = ESG_DIM;
  esgk::fill<esgk::kF32>(t);
  esgk::fill<esgk::kBF16>(t);
  esgk::fill<esgk::kFP8>(t);
  esgk::fill_scan<1>(t, 0);
  esgk::fill_scan<2>(t, 1);
  esgk::fill_scan<4>(t, 2);
  t->build_search[0] = esgk::kernel_ptr<esgk::kF32, 1, esgk::kBuildSearch>();
  t->build_search[1] = esgk::kernel_ptr<esgk::kF32, 2, esgk::kBuildSearch>();
  t->build_search[2] = esgk::kernel_ptr<esgk::kF32, 4, esgk::kBuildSearch>();
  t->build_search[3] = esgk::kernel_ptr<esgk::kF32, 8, esgk::kBuildSearch>();
  t->build_search[4] = esgk::kernel_ptr<esgk::kF32, 16, esgk::kBuildSearch>();
  using S32 = esgk::Shape<esgk::kF32>;
  t->build_prune = reinterpret_cast<const void*>(&esgk::build_prune_kernel<S32::G, S32::CPL>);
  t->build_reverse = reinterpret_cast<const void*>(&esgk::build_reverse_kernel<S32::G, S32::CPL>);
}
