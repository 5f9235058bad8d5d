// Device side of the index builder: the insertion rounds of Alg. 3 (and of
// the half-bounded index's chains, Alg. 2) on a HIP device.  The host
// builder (esg_build.cpp) plans the rounds, computes entry points and runs
// the reachability repair; these calls keep the vectors and the adjacency
// of every depth on the device and run, per round, the insertion searches,
// the occlusion pruning and the reverse edges there.  No HIP types appear
// here, so the host builder compiles without the HIP headers.
#pragma once

#include <cstdint>

namespace esgb {

struct GpuState;

// Device state on HIP device `device` for n rows of d float32 values
// (position order, copied from the host array X) and n_depth adjacency
// depths of R slots, all ESG_NO_NODE; insertion searches use beam width
// efc.  Rounds hold at most max_round points.  Errors: EINVAL,
// EUNSUPPORTED (no kernels for d, efc > ESG_EF_MAX), ENOMEM, EHIP.
int32_t gpu_open(int32_t device, const float* X, int64_t n, int32_t d, int32_t R,
                 int32_t n_depth, int32_t efc, int64_t max_round, GpuState** out);

// Replaces the device rows by X and empties every adjacency depth.
int32_t gpu_reset(GpuState* g, const float* X);

// Copies the adjacency rows [a, a + count) of depth src to depth dst.
int32_t gpu_copy_rows(GpuState* g, int32_t dst, int32_t src, int64_t a, int64_t count);

// One insertion round at `depth`: point pts[i] joins the graph on
// positions [lo[i], hi[i]] (searched from eps[i] against the graph as it
// was before the round), with at most R occlusion-pruned forward edges and
// the reverse edges, which re-prune a full row.  Each graph's rows must
// hold positions of that graph only.  Errors: EINVAL, EHIP.
int32_t gpu_round(GpuState* g, int32_t depth, int64_t nb, const uint32_t* pts,
                  const uint32_t* eps, const uint32_t* lo, const uint32_t* hi);

// Adjacency of one depth between host ([n][R]) and device.
int32_t gpu_get_rows(GpuState* g, int32_t depth, uint32_t* rows);
int32_t gpu_put_rows(GpuState* g, int32_t depth, const uint32_t* rows);

void gpu_close(GpuState* g);

}  // namespace esgb
