// libesg host runtime: index loading, storage codecs, launch of the search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/esg.h"
#include "esg_dims.h"
#include "esg_dispatch.h"
#include "esg_format.h"
#include "esg_kernels.h"
#include "esg_build_impl.h"
#include "esg_gpu_build.h"
#include "esg_scan_impl.h"

#define ESG_DECLARE_DIM(d) extern "C" void esg_register_dim_##d(esgk::KernelTable*);
ESG_DIMS(ESG_DECLARE_DIM)
#undef ESG_DECLARE_DIM

namespace {

constexpr int kDefaultHashCap = 4096;

const std::vector<esgk::KernelTable>& kernel_tables() {
  static const std::vector<esgk::KernelTable> tables = [] {
    std::vector<esgk::KernelTable> t;
#define ESG_REGISTER_DIM(d)           \
  {                                   \
    esgk::KernelTable kt;             \
    std::memset(&kt, 0, sizeof(kt));  \
    esg_register_dim_##d(&kt);        \
    t.push_back(kt);                  \
  }
    ESG_DIMS(ESG_REGISTER_DIM)
#undef ESG_REGISTER_DIM
    return t;
  }();
  return tables;
}

// Test hook: ESG_FAULT_ALLOC_AT=n makes the n-th device allocation (1-based,
// counted per process) report failure.
int64_t g_alloc_count = 0;

hipError_t dev_alloc(void** p, size_t bytes) {
  g_alloc_count++;
  const char* env = std::getenv("ESG_FAULT_ALLOC_AT");
  if (env && std::atoll(env) == g_alloc_count) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

}  // namespace

struct esg_index {
  int device = 0;
  int64_t n = 0;
  int32_t d = 0, dp = 0, R = 0, leaf = 0, n_depth = 0, c_den = 2, fanout = 2, layout = 0;
  int32_t metric = 0, dq = 0;   // ESG_METRIC_*; values per query row
  double max_norm2 = 0.0;
  int64_t* row_base = nullptr;  // [n_depth] device: row of position p at depth t = row_base[t] + p
  float* vec = nullptr;
  uint16_t* vec16 = nullptr;
  uint8_t* vec8 = nullptr;
  float* scale8 = nullptr;
  uint32_t* adj = nullptr;
  uint32_t* ep = nullptr;
  int64_t* ext_id = nullptr;
  uint32_t* spill = nullptr;
  int64_t spill_words = 0, spill_slots = 0;
  uint32_t* counter = nullptr;
  float* mlp_pack = nullptr;    // the predictor's weights in the search kernel's layout
  // brute-force scan: norms and rounding statistics of the bfloat16 copy
  float* norm2 = nullptr;
  float* stats = nullptr;       // [0] max |x|, [1] max relative bfloat16 rounding error
  float maxnorm = 0.0f, delta_x = 0.0f;
  // reserved workspace (esg_index_reserve)
  int64_t res_queries = 0, res_windows = 0;
  int32_t* win_q = nullptr;
  int64_t* win_s = nullptr;
  int64_t* win_e = nullptr;
  int32_t* win_order = nullptr;
  int32_t* q_win0 = nullptr;
  int32_t* q_nwin = nullptr;
  int32_t* qlist = nullptr;
  int32_t* wide = nullptr;
  int32_t* counts = nullptr;    // [0] narrow, [1] wide, [2] fallback, [3..] bucket histogram
  int32_t* fb_list = nullptr;
  int32_t* part_ef = nullptr;   // [res_queries][2] beams chosen before the search
  uint64_t* cand = nullptr;      // [res_windows * 64] per-window candidate lists
  int nbuckets = 0, bucket_shift = 11;
  hipStream_t capture_stream = nullptr;
  struct GraphEntry {
    std::vector<uint8_t> key;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<GraphEntry> graphs;
  int cu_count = 0;
  int64_t device_bytes = 0;
  const esgk::KernelTable* kt = nullptr;
  std::vector<void*> allocations;

  int32_t alloc(void** p, size_t bytes) {
    if (dev_alloc(p, bytes) != hipSuccess) {
      *p = nullptr;
      (void)hipGetLastError();
      return ESG_ENOMEM;
    }
    allocations.push_back(*p);
    device_bytes += (int64_t)bytes;
    return ESG_OK;
  }
  void release() {
    for (auto& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    capture_stream = nullptr;
    for (void* p : allocations) (void)hipFree(p);
    allocations.clear();
  }
};

namespace {

__global__ void reset_counter_kernel(uint32_t* c) { *c = 0u; }

// Predictor weights for inference: W1 and W2 regrouped as [input/4][hidden
// unit][4] (each hidden unit's lane reads 16 consecutive bytes per step and
// the wave one contiguous kilobyte); every other block is copied as is.
__global__ void mlp_pack_kernel(const float* __restrict__ src, float* __restrict__ dst) {
  using namespace esgk;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kMlpParams) return;
  int from = j;
  if (j < kOffB1) {                       // W1: [c][h][e] <- W1[h][4c + e]
    const int t = j - kOffW1, c = t / (4 * kHidden), h = (t / 4) % kHidden, e = t % 4;
    from = kOffW1 + h * kFeat + 4 * c + e;
  } else if (j >= kOffW2 && j < kOffB2) { // W2: [c][h][e] <- W2[h][4c + e]
    const int t = j - kOffW2, c = t / (4 * kHidden), h = (t / 4) % kHidden, e = t % 4;
    from = kOffW2 + h * kHidden + 4 * c + e;
  }
  dst[j] = src[from];
}

// Learned beam width chosen before the search (probe_hops = 0): one wave
// per query runs Alg. 4, and for each graph part the network maps the
// part's selection features (log2 of its filter width and node size, their
// ratio, log2 of the query width, parts - 1; the probe-state features are
// 0) to y; the part's beam is ef' = clamp(ceil(2^(y + delta)), k, ef).
// Writes the features, y and ef' to feat_out when given; with no network
// only the features.
// Learned beam width chosen before the search (probe_hops = 0), one
// thread per query: Alg. 4's parts, then for each graph part the network
// maps its selection features (log2 of its filter width and node size,
// their ratio, log2 of the query width, parts - 1; the seven probe-state
// inputs are 0) to y, and the part's beam is ef' = clamp(ceil(2^(y +
// delta)), k, ef).  The weights (caller's layout) are staged once per
// workgroup in LDS and read as broadcasts, so 256 queries share one copy
// instead of every query reading all of them from the caches.  Writes the
// features, y and ef' to feat_out when given; with no network only the
// features.
__global__ __launch_bounds__(256) void predict_beams_kernel(esgk::SearchArgs A,
                                                            const float* __restrict__ params,
                                                            int32_t* part_ef) {
  using namespace esgk;
  __shared__ float W[kMlpParams];
  if (params)
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) W[i] = params[i];
  __syncthreads();
  const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= A.nq) return;
  const int64_t lq = A.l[qi], rq = A.r[qi];
  int np = 0;
  Part pt{};
  if (lq >= 0 && rq < A.n && lq <= rq) np = select_parts(A, lq, rq, 0, pt);
  for (int p = 0; p < 2; p++) {
    if (p == 1 && np == 2) select_parts(A, lq, rq, 1, pt);
    int efp = A.ef;
    if (p < np && pt.kind == 1) {
      const float wp = (float)(pt.y - pt.x + 1), L = (float)(pt.b - pt.a + 1);
      float f[5];
      f[0] = __log2f(wp);
      f[1] = __log2f(L);
      f[2] = wp / L;
      f[3] = __log2f((float)(rq - lq + 1));
      f[4] = (float)(np - 1);
      float y = 0.0f;
      if (params) {
        float x[kFeat];
#pragma unroll
        for (int i = 0; i < kFeat; i++)
          x[i] = ((i < 5 ? f[i] : 0.0f) - W[kOffMu + i]) / W[kOffSd + i];
        float h[kHidden];
#pragma unroll
        for (int j = 0; j < kHidden; j++) {
          float a = W[kOffB1 + j];
#pragma unroll
          for (int i = 0; i < kFeat; i++) a = __builtin_fmaf(W[kOffW1 + j * kFeat + i], x[i], a);
          h[j] = a > 0.0f ? a : 0.0f;
          __builtin_amdgcn_sched_barrier(0);   // keeps the weight reads of one unit together
        }
        y = W[kOffB3];
        for (int j = 0; j < kHidden; j++) {
          float a = W[kOffB2 + j];
#pragma unroll
          for (int i = 0; i < kHidden; i++) {
            a = __builtin_fmaf(W[kOffW2 + j * kHidden + i], h[i], a);
            if ((i & 15) == 15) __builtin_amdgcn_sched_barrier(0);
          }
          y = __builtin_fmaf(W[kOffW3 + j], a > 0.0f ? a : 0.0f, y);
        }
        const float e2 = exp2f(y + A.mlp_delta);
        efp = e2 >= (float)A.ef ? A.ef : (int)ceilf(e2);
        efp = efp < A.k ? A.k : efp;
      }
      if (A.feat_out) {
        float* out = A.feat_out + (qi * 2 + p) * kFeatStride;
        for (int i = 0; i < kFeat; i++) out[i] = i < 5 ? f[i] : 0.0f;
        out[kFeat] = y;
        out[kFeat + 1] = (float)efp;
      }
    }
    if (part_ef) part_ef[qi * 2 + p] = efp;
  }
}

// float32 -> bfloat16, round to nearest even (finite inputs).
__global__ void encode_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y,
                                   int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t b = __float_as_uint(x[i]);
    b += 0x7FFFu + ((b >> 16) & 1u);
    y[i] = (uint16_t)(b >> 16);
  }
}

// |y| -> OCP E4M3 code (no sign): nearest, ties to even, saturating at 448.
__device__ uint32_t e4m3_magnitude_code(float a) {
  a = fminf(a, 448.0f);
  if (a < 0.015625f) {                       // below 2^-6: subnormal step 2^-9
    return (uint32_t)__builtin_rintf(a * 512.0f);
  }
  uint32_t b = __float_as_uint(a);
  b += 0x7FFFFu + ((b >> 20) & 1u);          // round to 3 mantissa bits
  uint32_t e = (b >> 23) - 120u;             // float exponent -> e4m3 exponent
  uint32_t code = (e << 3) | ((b >> 20) & 7u);
  return code > 126u ? 126u : code;
}

// One wave per row: scale = max|x| / 448 (1 for a zero row), codes of x/scale.
__global__ void encode_fp8_kernel(const float* __restrict__ x, int64_t n, int32_t d, int32_t dp,
                                  uint8_t* __restrict__ y, float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n) return;
  const float* xr = x + row * dp;
  float m = 0.0f;
  for (int j = lane; j < d; j += 64) m = fmaxf(m, fabsf(xr[j]));
  for (int s = 32; s >= 1; s >>= 1) m = fmaxf(m, __shfl_xor(m, s));
  float sc = m / 448.0f;
  if (!(sc > 0.0f)) sc = 1.0f;
  if (lane == 0) scale[row] = sc;
  uint8_t* yr = y + row * dp;
  for (int j = lane; j < dp; j += 64) {
    uint32_t code = 0u;
    if (j < d) {
      float v = xr[j] / sc;
      code = e4m3_magnitude_code(fabsf(v));
      if (v < 0.0f && code != 0u) code |= 0x80u;
    }
    yr[j] = (uint8_t)code;
  }
}

// |x|^2 per row (float32), the largest |x| and the largest relative
// bfloat16 rounding error of any element.  One wave per row (grid-stride
// over the rows); each workgroup reduces its waves' maxima in LDS and adds
// one pair of atomics (per-row atomics to the same two words serialised
// the kernel).
__global__ __launch_bounds__(256) void norms_kernel(const float* __restrict__ x,
                                                    const uint16_t* __restrict__ xb, int64_t n,
                                                    int32_t d, int32_t dp, float* __restrict__ norm2,
                                                    float* __restrict__ stats) {
  const int lane = threadIdx.x & 63;
  const int wib = (int)(threadIdx.x >> 6), wpb = (int)(blockDim.x >> 6);
  float mx = 0.0f, rmax = 0.0f;
  for (int64_t row = (int64_t)blockIdx.x * wpb + wib; row < n; row += (int64_t)gridDim.x * wpb) {
    float s = 0.0f, rel = 0.0f;
    for (int j = lane; j < d; j += 64) {
      const float v = x[row * dp + j];
      s = __builtin_fmaf(v, v, s);
      const float vb = __uint_as_float((uint32_t)xb[row * dp + j] << 16);
      if (v != 0.0f) rel = fmaxf(rel, fabsf(vb - v) / fabsf(v));
    }
    for (int m = 32; m >= 1; m >>= 1) {
      s += __shfl_xor(s, m);
      rel = fmaxf(rel, __shfl_xor(rel, m));
    }
    if (lane == 0) norm2[row] = s;
    mx = fmaxf(mx, sqrtf(s));
    rmax = fmaxf(rmax, rel);
  }
  __shared__ float smx[4], srel[4];
  if (lane == 0) {
    smx[wib] = mx;
    srel[wib] = rmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = 0.0f, b = 0.0f;
    for (int w = 0; w < wpb; w++) {
      a = fmaxf(a, smx[w]);
      b = fmaxf(b, srel[w]);
    }
    atomicMax(reinterpret_cast<unsigned int*>(stats), __float_as_uint(a));
    atomicMax(reinterpret_cast<unsigned int*>(stats) + 1, __float_as_uint(b));
  }
}

__global__ void zero_i32_kernel(int32_t* p, int32_t count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0;
}

// Router: queries narrower than `thr` become one scan window each; the rest
// (and invalid ranges) go to the graph search list.
__global__ void classify_kernel(const int64_t* __restrict__ l, const int64_t* __restrict__ r,
                                int64_t nq, int64_t n, int64_t thr, int32_t* win_q,
                                int64_t* win_s, int64_t* win_e, int32_t* q_win0,
                                int32_t* q_nwin, int32_t* wide, int32_t* counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const int64_t a = l[i], b = r[i];
  const bool valid = a >= 0 && b < n && a <= b;
  if (valid && b - a + 1 < thr) {
    const int32_t slot = atomicAdd(&counts[0], 1);
    win_q[slot] = (int32_t)i;
    win_s[slot] = a;
    win_e[slot] = b;
    q_win0[i] = slot;
    q_nwin[i] = 1;
  } else {
    const int32_t slot = atomicAdd(&counts[1], 1);
    wide[slot] = (int32_t)i;
  }
}

__global__ void bucket_hist_kernel(const int64_t* __restrict__ win_s, const int32_t* counts,
                                   int32_t shift, int32_t* hist) {
  const int64_t nw = counts[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
       i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&hist[win_s[i] >> shift], 1);
}

// Exclusive prefix sum of nb <= 1024 bucket counts, in place (one block).
__global__ void bucket_scan_kernel(int32_t* hist, int32_t nb) {
  __shared__ int32_t buf[1024];
  const int t = threadIdx.x;
  buf[t] = t < nb ? hist[t] : 0;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t v = t >= off ? buf[t - off] : 0;
    __syncthreads();
    buf[t] += v;
    __syncthreads();
  }
  if (t < nb) hist[t] = buf[t] - (t < nb ? hist[t] : 0);
}

__global__ void bucket_scatter_kernel(const int64_t* __restrict__ win_s, const int32_t* counts,
                                      int32_t shift, int32_t* cursor, int32_t* order) {
  const int64_t nw = counts[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t pos = atomicAdd(&cursor[win_s[i] >> shift], 1);
    order[pos] = (int32_t)i;
  }
}

bool read_exact(FILE* f, uint64_t off, void* dst, uint64_t bytes) {
  if (fseeko(f, (off_t)off, SEEK_SET) != 0) return false;
  char* c = static_cast<char*>(dst);
  while (bytes > 0) {
    size_t chunk = (size_t)std::min<uint64_t>(bytes, 1ull << 30);
    if (fread(c, 1, chunk, f) != chunk) return false;
    c += chunk;
    bytes -= chunk;
  }
  return true;
}

// Chain layout: every recorded prefix or suffix graph has its entry and all
// neighbours of its rows inside its own range.
bool chains_are_consistent(int64_t n, const std::vector<int64_t>& sizes, int32_t R,
                           const std::vector<int64_t>& row_base, const uint32_t* adj,
                           const uint32_t* ep) {
  const size_t k = sizes.size();
  for (size_t t = 0; t < 2 * k; t++) {
    const int64_t sz = sizes[t % k], a = t < k ? 0 : n - sz, b = a + sz - 1;
    const uint32_t e = ep[t + 1];
    if (e == ESG_NO_NODE || (int64_t)e < a || (int64_t)e > b) return false;
    for (int64_t p = a; p <= b; p++)
      for (int32_t j = 0; j < R; j++) {
        const uint32_t v = adj[(size_t)(row_base[t] + p) * R + j];
        if (v != ESG_NO_NODE && ((int64_t)v < a || (int64_t)v > b)) return false;
      }
  }
  return true;
}

bool tree_is_consistent(int64_t n, int32_t leaf, int32_t fanout, int32_t n_depth, int32_t R,
                        const uint32_t* adj, const uint32_t* ep) {
  struct Node {
    int64_t a, b, heap;
    int32_t depth;
  };
  std::vector<Node> todo{{0, n - 1, 1, 0}};
  while (!todo.empty()) {
    Node nd = todo.back();
    todo.pop_back();
    if (nd.b - nd.a < leaf) continue;
    if (nd.depth >= n_depth) return false;
    const uint32_t e = ep[nd.heap];
    if (e == ESG_NO_NODE || (int64_t)e < nd.a || (int64_t)e > nd.b) return false;
    const uint32_t* rows = adj + (size_t)nd.depth * (size_t)n * (size_t)R;
    for (int64_t p = nd.a; p <= nd.b; p++)
      for (int32_t j = 0; j < R; j++) {
        const uint32_t v = rows[(size_t)p * R + j];
        if (v != ESG_NO_NODE && ((int64_t)v < nd.a || (int64_t)v > nd.b)) return false;
      }
    const int64_t L = nd.b - nd.a + 1;
    for (int64_t j = 0; j < fanout; j++) {
      const int64_t ca = nd.a + (j * L + fanout - 1) / fanout;
      const int64_t cb = nd.a + ((j + 1) * L + fanout - 1) / fanout - 1;
      if (ca <= cb) todo.push_back({ca, cb, (int64_t)fanout * (nd.heap - 1) + 2 + j, nd.depth + 1});
    }
  }
  return true;
}

// Lanes per vector for C chunks: the next power of two, at most a wave.
int lanes_for_chunks(int64_t c) {
  int g = 1;
  while (g < c) g *= 2;
  return g > 64 ? 64 : g;
}

// A kernel table compiled for dimension cls serves dimension d when every
// storage type (4, 8, 16 values per 16-byte chunk) has the same lanes per
// vector and chunks per lane, and d's padded row fits cls's.
bool same_shape(int64_t d, int64_t cls) {
  for (int w : {4, 8, 16}) {
    const int64_t c = (d + w - 1) / w, cc = (cls + w - 1) / w;
    const int g = lanes_for_chunks(c), gc = lanes_for_chunks(cc);
    if (g != gc || (c + g - 1) / g != (cc + gc - 1) / gc) return false;
  }
  return (d + 15) / 16 <= (cls + 15) / 16;
}

int width_index(int cap) {
  if (cap <= 64) return 0;
  if (cap <= 128) return 1;
  if (cap <= 256) return 2;
  if (cap <= 512) return 3;
  return 4;
}

// Host-to-device copies of index data go through a pinned staging buffer
// that the library allocates once (hipHostMalloc) and keeps: large copies
// straight from pageable memory have left device data that did not match
// its source (seen right after a device build in the same process, under
// the kernel tracer).  Rows of `width` bytes (source pitch spitch) land in
// device rows of dpitch bytes whose tail is zero-filled in the staging
// buffer.  Synchronous; false on a HIP error.
std::mutex g_stage_mu;
char* g_stage = nullptr;
constexpr size_t kStagingBytes = (size_t)64 << 20;

bool h2d_rows(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
              size_t rows) {
  if (rows == 0 || width == 0) return true;
  std::lock_guard<std::mutex> lock(g_stage_mu);
  if (!g_stage && hipHostMalloc((void**)&g_stage, kStagingBytes, hipHostMallocDefault) != hipSuccess) {
    g_stage = nullptr;
    return false;
  }
  if (dpitch > kStagingBytes) return false;
  const size_t per = kStagingBytes / dpitch;   // rows per chunk
  for (size_t r0 = 0; r0 < rows; r0 += per) {
    const size_t nr = std::min(per, rows - r0);
    for (size_t r = 0; r < nr; r++) {
      std::memcpy(g_stage + r * dpitch, static_cast<const char*>(src) + (r0 + r) * spitch, width);
      if (dpitch > width) std::memset(g_stage + r * dpitch + width, 0, dpitch - width);
    }
    if (hipMemcpy(static_cast<char*>(dst) + r0 * dpitch, g_stage, nr * dpitch,
                  hipMemcpyHostToDevice) != hipSuccess)
      return false;
  }
  return true;
}

bool h2d(void* dst, const void* src, size_t bytes) {
  const size_t chunk = (size_t)1 << 20;   // rows of 1 MB and a last row with the rest
  const size_t full = bytes / chunk, rest = bytes - full * chunk;
  const char* s = static_cast<const char*>(src) + full * chunk;
  return h2d_rows(dst, chunk, src, chunk, chunk, full) &&
         h2d_rows(static_cast<char*>(dst) + full * chunk, rest, s, rest, rest, rest ? 1 : 0);
}

// Checksum of an upload: the 64-bit sum over words i of mix(i, word i),
// order-independent, so the device adds it up in any order.
__host__ __device__ inline uint64_t mix_word(uint64_t i, uint32_t w) {
  uint64_t x = ((uint64_t)w | (i << 32)) ^ (i >> 32);
  x *= 0x9E3779B97F4A7C15ull;
  return x ^ (x >> 29);
}

__global__ void checksum_kernel(const uint32_t* __restrict__ p, uint64_t n,
                                unsigned long long* __restrict__ out) {
  uint64_t s = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    s += mix_word(i, p[i]);
  __shared__ unsigned long long part[256];
  part[threadIdx.x] = s;
  __syncthreads();
  for (unsigned w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, part[0]);
}

// Test hook: ESG_FAULT_UPLOAD_CHECK=n makes the n-th upload check (1-based,
// counted per process) report a difference, =all every check.
std::atomic<int64_t> g_check_count{0};

bool upload_check_forced() {
  const int64_t c = ++g_check_count;
  const char* env = std::getenv("ESG_FAULT_UPLOAD_CHECK");
  return env && (std::strcmp(env, "all") == 0 || std::atoll(env) == c);
}

// Compares a device copy with its host source: rows of `width` 32-bit words
// on the host land in device rows of `pitch` words whose tail is zero.
// Returns 1 when they match, 0 when they differ, -1 on a HIP error.
int verify_upload(const void* dev, const void* host, int64_t rows, int64_t width, int64_t pitch) {
  const bool forced = upload_check_forced();
  const uint32_t* h = static_cast<const uint32_t*>(host);
  const int nt = 8;
  uint64_t part[nt] = {0};
  std::vector<std::thread> th;
  for (int t = 0; t < nt; t++)
    th.emplace_back([&, t] {
      uint64_t s = 0;
      for (int64_t r = rows * t / nt; r < rows * (t + 1) / nt; r++)
        for (int64_t j = 0; j < pitch; j++)
          s += mix_word((uint64_t)(r * pitch + j), j < width ? h[r * width + j] : 0u);
      part[t] = s;
    });
  for (auto& x : th) x.join();
  uint64_t want = 0;
  for (int t = 0; t < nt; t++) want += part[t];
  unsigned long long* d = nullptr;
  unsigned long long got = 0;
  const bool ok = hipMalloc((void**)&d, 8) == hipSuccess && hipMemset(d, 0, 8) == hipSuccess &&
                  (checksum_kernel<<<1024, 256>>>(static_cast<const uint32_t*>(dev),
                                                  (uint64_t)(rows * pitch), d),
                   hipGetLastError() == hipSuccess) &&
                  hipMemcpy(&got, d, 8, hipMemcpyDeviceToHost) == hipSuccess;
  if (d) (void)hipFree(d);
  if (!ok) {
    (void)hipGetLastError();
    return -1;
  }
  return got == want && !forced ? 1 : 0;
}

int32_t load_impl(const char* path, int32_t hip_device, esg_index** out) {
  FILE* f = fopen(path, "rb");
  if (!f) return ESG_EIO;
  struct Closer {
    FILE* f;
    ~Closer() { fclose(f); }
  } closer{f};

  esg::FileHeader h;
  if (fread(&h, 1, sizeof(h), f) != sizeof(h)) return ESG_EFORMAT;
  const esg::Crc32c& crc = esg::crc32c();
  if (std::memcmp(h.magic, esg::kMagic, 8) != 0 || h.version != esg::kVersion ||
      h.header_bytes != esg::kHeaderBytes)
    return ESG_EFORMAT;
  if (crc.update(0, &h, offsetof(esg::FileHeader, crc_header)) != h.crc_header) return ESG_EFORMAT;
  if (h.n <= 0 || h.n >= (int64_t)ESG_NO_NODE || h.d <= 0 || h.d > 65536 || h.degree < 1 ||
      h.degree > ESG_DEGREE_MAX || h.leaf < 1 || h.fanout < 2 || h.fanout > ESG_FANOUT_MAX ||
      h.n_depth < 0 || h.n_depth > 40 || h.c_den < h.fanout || h.layout < 0 || h.layout > 1 ||
      (h.layout == 0 && esg::ep_count(h.n_depth, h.fanout) == 0))
    return ESG_EFORMAT;   // c = 1/c_den <= 1/fanout keeps Alg. 4 at two parts at most
  if (h.metric < ESG_METRIC_L2 || h.metric > ESG_METRIC_IP ||
      h.dq != (h.metric == ESG_METRIC_IP ? h.d - 1 : h.d) || h.dq < 1 ||
      !(h.max_norm2 >= 0.0 && h.max_norm2 <= 1e300) ||
      (h.metric != ESG_METRIC_IP && h.max_norm2 != 0.0))
    return ESG_EFORMAT;
  // rows per depth: the tree's depths cover all n positions; the chains'
  // depths only their own prefix or suffix
  std::vector<int64_t> row_base((size_t)h.n_depth);
  uint64_t adj_rows = (uint64_t)h.n_depth * (uint64_t)h.n, ep_slots = 0;
  std::vector<int64_t> chain;
  if (h.layout == 1) {
    chain = esg::chain_sizes(h.n, h.leaf, h.fanout);
    if ((int64_t)h.n_depth != 2 * (int64_t)chain.size()) return ESG_EFORMAT;
    row_base = esg::chain_row_base(h.n, chain);
    adj_rows = (uint64_t)esg::chain_rows(chain);
    ep_slots = (uint64_t)h.n_depth + 1;
  } else {
    for (int32_t t = 0; t < h.n_depth; t++) row_base[(size_t)t] = (int64_t)t * h.n;
    ep_slots = esg::ep_count(h.n_depth, h.fanout);
  }
  const uint64_t sizes[5] = {esg::bytes_ids(h.n), esg::bytes_attr(h.n), esg::bytes_vec(h.n, h.d),
                             adj_rows * (uint64_t)h.degree * 4, ep_slots * 4};
  const uint64_t offs[5] = {h.off_ids, h.off_attr, h.off_vec, h.off_adj, h.off_ep};
  uint64_t prev_end = esg::kHeaderBytes;
  for (int s = 0; s < 5; s++) {
    if (offs[s] < prev_end || offs[s] % esg::kAlign != 0) return ESG_EFORMAT;
    prev_end = offs[s] + sizes[s];
  }
  if (fseeko(f, 0, SEEK_END) != 0) return ESG_EIO;
  const uint64_t fsize = (uint64_t)ftello(f);
  if (prev_end != h.file_bytes || fsize != h.file_bytes) return ESG_EFORMAT;
  if (h.degree > esgk::kBatch) return ESG_EUNSUPPORTED;

  const esgk::KernelTable* kt = nullptr;
  for (const auto& t : kernel_tables())
    if (!kt && same_shape(h.d, t.dim)) kt = &t;
  if (!kt) return ESG_EUNSUPPORTED;

  std::vector<int64_t> ids((size_t)h.n);
  std::vector<float> vec((size_t)h.n * (size_t)h.d);
  std::vector<uint32_t> adj((size_t)adj_rows * (size_t)h.degree);
  std::vector<uint32_t> ep((size_t)ep_slots);
  std::vector<double> attr((size_t)h.n);
  void* dsts[5] = {ids.data(), attr.data(), vec.data(), adj.data(), ep.data()};
  for (int s = 0; s < 5; s++) {
    if (!read_exact(f, offs[s], dsts[s], sizes[s])) return ESG_EIO;
    if (crc.update(0, dsts[s], sizes[s]) != h.crc_sections[s]) return ESG_EFORMAT;
  }
  // Structural checks the kernels rely on: every graph node [a,b] of the
  // tree has its entry point and all neighbours of its rows inside [a,b].
  if (h.layout == 1 ? !chains_are_consistent(h.n, chain, h.degree, row_base, adj.data(), ep.data())
                    : !tree_is_consistent(h.n, h.leaf, h.fanout, h.n_depth, h.degree, adj.data(),
                                          ep.data()))
    return ESG_EFORMAT;

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return ESG_EHIP;
  }
  if (hip_device < 0 || hip_device >= ndev) return ESG_EINVAL;
  if (hipSetDevice(hip_device) != hipSuccess) return ESG_EHIP;

  esg_index* ix = new (std::nothrow) esg_index();
  if (!ix) return ESG_ENOMEM;
  ix->device = hip_device;
  ix->n = h.n;
  ix->d = h.d;
  ix->dp = (h.d + 15) / 16 * 16;
  ix->R = h.degree;
  ix->leaf = h.leaf;
  ix->n_depth = h.n_depth;
  ix->c_den = h.c_den;
  ix->fanout = h.fanout;
  ix->layout = h.layout;
  ix->metric = h.metric;
  ix->dq = h.dq;
  ix->max_norm2 = h.max_norm2;
  ix->kt = kt;
  if (hipDeviceGetAttribute(&ix->cu_count, hipDeviceAttributeMultiprocessorCount, hip_device) !=
      hipSuccess) {
    delete ix;
    return ESG_EHIP;
  }
  ix->spill_slots = (int64_t)ix->cu_count * 32;
  ix->spill_words = ((h.n + 31) / 32 + 63) / 64 * 64;

  int32_t st = ESG_OK;
  auto A = [&](void** p, size_t b) {
    if (st == ESG_OK) st = ix->alloc(p, b);
  };
  A((void**)&ix->vec, (size_t)h.n * ix->dp * 4);
  A((void**)&ix->adj, std::max<size_t>(4, adj.size() * 4));
  A((void**)&ix->ep, ep.size() * 4);
  A((void**)&ix->ext_id, ids.size() * 8);
  const size_t spill_bytes = (size_t)ix->spill_slots * (ix->spill_words + esgk::kSpillLog) * 4;
  A((void**)&ix->spill, spill_bytes);
  A((void**)&ix->counter, 256);
  A((void**)&ix->mlp_pack, sizeof(float) * esgk::kMlpParams);
  A((void**)&ix->row_base, std::max<size_t>(8, row_base.size() * 8));
  if (st != ESG_OK) {
    ix->release();
    delete ix;
    return st;
  }
  // rows are padded with zeros to dp values on the way
  auto upload = [&]() {
    return h2d_rows(ix->vec, (size_t)ix->dp * 4, vec.data(), (size_t)h.d * 4, (size_t)h.d * 4,
                    (size_t)h.n) &&
           h2d(ix->adj, adj.data(), adj.size() * 4) && h2d(ix->ep, ep.data(), ep.size() * 4) &&
           h2d(ix->row_base, row_base.data(), row_base.size() * 8) &&
           h2d(ix->ext_id, ids.data(), ids.size() * 8) &&
           hipMemset(ix->counter, 0, 256) == hipSuccess &&
           hipMemset(ix->spill, 0, spill_bytes) == hipSuccess &&   // bitmaps start all zero
           hipDeviceSynchronize() == hipSuccess;
  };
  // The device copies of the vectors and the adjacency are checked against
  // the (checksummed) file contents once everything is in place; a copy
  // that differs is made again once, and a second difference is an error.
  auto verified = [&]() {
    const int v = verify_upload(ix->vec, vec.data(), h.n, h.d, ix->dp);
    const int a = adj.empty() ? 1
                              : verify_upload(ix->adj, adj.data(), (int64_t)adj.size() / h.degree,
                                              h.degree, h.degree);
    return v < 0 || a < 0 ? -1 : (v == 1 && a == 1 ? 1 : 0);
  };
  bool ok = upload();
  int check = ok ? verified() : -1;
  if (check == 0) {
    std::fprintf(stderr, "esg_load_index: the device copy of %s differs from the file; copying "
                 "again\n", path);
    ok = upload();
    check = ok ? verified() : -1;
    if (check == 0)
      std::fprintf(stderr, "esg_load_index: the device copy of %s differs again\n", path);
  }
  ok = ok && check == 1;
  if (!ok) {
    (void)hipGetLastError();
    ix->release();
    delete ix;
    return ESG_EHIP;
  }
  *out = ix;
  return ESG_OK;
}

}  // namespace

extern "C" {

const char* esg_status_str(int32_t s) {
  switch (s) {
    case ESG_OK: return "ESG_OK";
    case ESG_EINVAL: return "ESG_EINVAL: invalid argument";
    case ESG_ERANGE: return "ESG_ERANGE: value out of the supported range";
    case ESG_ENOMEM: return "ESG_ENOMEM: allocation failed";
    case ESG_EIO: return "ESG_EIO: file I/O failed";
    case ESG_EFORMAT: return "ESG_EFORMAT: malformed index file";
    case ESG_EHIP: return "ESG_EHIP: HIP runtime error";
    case ESG_EUNSUPPORTED: return "ESG_EUNSUPPORTED: unsupported for this index";
    case ESG_EOVERFLOW: return "ESG_EOVERFLOW: device structure overflow";
    default: return "ESG: unknown status";
  }
}

int32_t esg_load_index(const char* path, int32_t hip_device, esg_index** out) {
  if (!path || !out) return ESG_EINVAL;
  *out = nullptr;
  try {
    return load_impl(path, hip_device, out);
  } catch (const std::bad_alloc&) {
    return ESG_ENOMEM;
  } catch (...) {
    return ESG_EINVAL;
  }
}

void esg_free_index(esg_index* idx) {
  if (!idx) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(idx->device);
  (void)hipDeviceSynchronize();
  idx->release();
  (void)hipSetDevice(cur);
  delete idx;
}

int32_t esg_index_info(const esg_index* idx, esg_index_info_t* out) {
  if (!idx || !out) return ESG_EINVAL;
  out->n = idx->n;
  out->d = idx->d;
  out->degree = idx->R;
  out->leaf = idx->leaf;
  out->fanout = idx->fanout;
  out->n_depth = idx->n_depth;
  out->c_den = idx->c_den;
  out->has_bf16 = idx->vec16 != nullptr;
  out->has_fp8 = idx->vec8 != nullptr;
  out->device_bytes = idx->device_bytes;
  out->metric = idx->metric;
  out->dq = idx->dq;
  out->max_norm2 = idx->max_norm2;
  return ESG_OK;
}

int32_t esg_index_copy_storage(const esg_index* idx, int32_t kind, void* dst, int64_t bytes) {
  if (!idx || !dst || kind < 0 || kind > 2) return ESG_EINVAL;
  const int64_t n = idx->n, d = idx->d, dp = idx->dp;
  const int64_t esz = kind == 0 ? 4 : kind == 1 ? 2 : 1;
  const int64_t want = n * d * esz + (kind == 2 ? n * 4 : 0);
  if (bytes != want) return ESG_EINVAL;
  const void* src = kind == 0 ? (const void*)idx->vec
                  : kind == 1 ? (const void*)idx->vec16 : (const void*)idx->vec8;
  if (!src) return ESG_EUNSUPPORTED;
  if (hipSetDevice(idx->device) != hipSuccess) return ESG_EHIP;
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy2D(dst, (size_t)(d * esz), src, (size_t)(dp * esz), (size_t)(d * esz), (size_t)n,
                  hipMemcpyDeviceToHost) != hipSuccess)
    return ESG_EHIP;
  if (kind == 2 && hipMemcpy(static_cast<char*>(dst) + n * d, idx->scale8, (size_t)n * 4,
                             hipMemcpyDeviceToHost) != hipSuccess)
    return ESG_EHIP;
  return ESG_OK;
}

int32_t esg_index_add_storage(esg_index* idx, int32_t kind, void* stream) {
  if (!idx || (kind != ESG_TRAV_BF16 && kind != ESG_TRAV_FP8)) return ESG_EINVAL;
  if (hipSetDevice(idx->device) != hipSuccess) return ESG_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t count = idx->n * idx->dp;
  if (kind == ESG_TRAV_BF16) {
    if (idx->vec16) return ESG_OK;
    int32_t st = idx->alloc((void**)&idx->vec16, (size_t)count * 2);
    if (st == ESG_OK) st = idx->alloc((void**)&idx->norm2, (size_t)idx->n * 4);
    if (st == ESG_OK) st = idx->alloc((void**)&idx->stats, 256);
    if (st != ESG_OK) return st;
    encode_bf16_kernel<<<4096, 256, 0, s>>>(idx->vec, idx->vec16, count);
    zero_i32_kernel<<<1, 64, 0, s>>>(reinterpret_cast<int32_t*>(idx->stats), 64);
    norms_kernel<<<(unsigned)std::min<int64_t>(2048, (idx->n + 3) / 4), 256, 0, s>>>(
        idx->vec, idx->vec16, idx->n, idx->d, idx->dp, idx->norm2, idx->stats);
    float host_stats[2] = {0.0f, 0.0f};
    if (hipMemcpyAsync(host_stats, idx->stats, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return ESG_EHIP;
    idx->maxnorm = host_stats[0];
    idx->delta_x = host_stats[1];
  } else {
    if (idx->vec8) return ESG_OK;
    int32_t st = idx->alloc((void**)&idx->vec8, (size_t)count);
    if (st == ESG_OK) st = idx->alloc((void**)&idx->scale8, (size_t)idx->n * 4);
    if (st != ESG_OK) return st;
    const int64_t blocks = (idx->n + 3) / 4;
    encode_fp8_kernel<<<(unsigned)blocks, 256, 0, s>>>(idx->vec, idx->n, idx->d, idx->dp,
                                                       idx->vec8, idx->scale8);
  }
  if (hipGetLastError() != hipSuccess) return ESG_EHIP;
  return ESG_OK;
}

int32_t esg_index_reserve(esg_index* idx, int64_t max_queries, int64_t max_windows) {
  if (!idx || max_queries < 1 || max_windows < 1 || max_queries > 0x7FFFFFFF ||
      max_windows > 0x7FFFFFFF)
    return ESG_EINVAL;
  if (max_queries <= idx->res_queries && max_windows <= idx->res_windows) return ESG_OK;
  if (idx->res_queries > 0) return ESG_EINVAL;  // one reservation per index
  if (hipSetDevice(idx->device) != hipSuccess) return ESG_EHIP;
  int shift = 11;
  while (((idx->n - 1) >> shift) + 1 > 1024) shift++;
  idx->bucket_shift = shift;
  idx->nbuckets = (int)(((idx->n - 1) >> shift) + 1);
  const size_t Q = (size_t)max_queries, W = (size_t)std::max(max_windows, max_queries);
  int32_t st = ESG_OK;
  auto A = [&](void** p, size_t b) {
    if (st == ESG_OK) st = idx->alloc(p, b);
  };
  A((void**)&idx->win_q, W * 4);
  A((void**)&idx->win_s, W * 8);
  A((void**)&idx->win_e, W * 8);
  A((void**)&idx->win_order, W * 4);
  A((void**)&idx->q_win0, Q * 4);
  A((void**)&idx->q_nwin, Q * 4);
  A((void**)&idx->qlist, Q * 4);
  A((void**)&idx->wide, Q * 4);
  A((void**)&idx->fb_list, Q * 4);
  A((void**)&idx->part_ef, Q * 8);
  A((void**)&idx->counts, (size_t)(4 + idx->nbuckets) * 4);
  A((void**)&idx->cand, W * 64 * 8);
  if (st != ESG_OK) return st;
  if (hipStreamCreateWithFlags(&idx->capture_stream, hipStreamNonBlocking) != hipSuccess)
    return ESG_EHIP;
  idx->res_queries = (int64_t)Q;
  idx->res_windows = (int64_t)W;
  return ESG_OK;
}

namespace {

int scan_width_index(int k) { return k <= 32 ? 0 : (k <= 64 ? 1 : 2); }

esgk::ScanArgs scan_args(esg_index* idx, const float* queries, const int64_t* l, const int64_t* r,
                         int64_t nq, int32_t k, int32_t mr, int64_t* ids, float* dists,
                         int32_t* certified) {
  esgk::ScanArgs S;
  std::memset(&S, 0, sizeof(S));
  S.vec = idx->vec;
  S.vec16 = idx->vec16;
  S.norm2 = idx->norm2;
  S.ext_id = idx->ext_id;
  S.n = idx->n;
  S.d = idx->d;
  S.dq = idx->dq;
  S.dp = idx->dp;
  S.queries = queries;
  S.l = l;
  S.r = r;
  S.nq = nq;
  S.k = k;
  S.mr = mr;
  S.win_q = idx->win_q;
  S.win_s = idx->win_s;
  S.win_e = idx->win_e;
  S.win_order = idx->win_order;
  S.q_win0 = idx->q_win0;
  S.q_nwin = idx->q_nwin;
  S.cand = idx->cand;
  S.cand_stride = 64 << scan_width_index(k);
  S.ids = ids;
  S.dists = dists;
  S.fb_list = idx->fb_list;
  S.fb_count = idx->counts + 2;
  S.certified = certified;
  S.delta_x = idx->delta_x;
  S.maxnorm = idx->maxnorm;
  S.gamma = (float)(idx->d + 4) * 5.9604645e-8f;
  S.g_rel = 1.0f / 65536.0f;
  return S;
}

int32_t launch_fn(const void* fn, int64_t grid, size_t lds, void* arg, hipStream_t s) {
  if (grid <= 0) return ESG_OK;
  void* args[] = {arg};
  if (hipLaunchKernel(fn, dim3((unsigned)grid), dim3(256), args, lds, s) != hipSuccess) {
    (void)hipGetLastError();
    return ESG_EHIP;
  }
  return ESG_OK;
}

// The scan kernels over windows already described in the workspace.
int32_t launch_scan(esg_index* idx, esgk::ScanArgs& S, int64_t nw_bound, int64_t nq_bound,
                    hipStream_t s) {
  const int wi = scan_width_index(S.k);
  int32_t st = launch_fn(idx->kt->scan_select[wi], (nw_bound + 63) / 64, 0, &S, s);
  if (st == ESG_OK)
    st = launch_fn(idx->kt->rerank[wi], (nq_bound + 3) / 4, 4 * esgk::kStageBytes, &S, s);
  // fallback: the window pass takes every resident wave slot (the windows of
  // the few uncertified queries are spread over all of them)
  if (st == ESG_OK)
    st = launch_fn(idx->kt->fallback[wi], std::min<int64_t>(4 * (int64_t)idx->cu_count,
                                                          (nw_bound + 3) / 4),
                   4 * esgk::kStageBytes, &S, s);
  if (st == ESG_OK)
    st = launch_fn(idx->kt->fb_merge[wi], std::min<int64_t>(1024, (nq_bound + 3) / 4), 0, &S, s);
  return st;
}

}  // namespace

namespace {

// ---- 0. windows on the device --------------------------------------------------
// Query i (listed in qlist) owns windows q_win0[i] .. + q_nwin[i] - 1 (the
// host computed both); window j covers [l + j kWin, min(r, l + (j+1) kWin - 1)].
__global__ void scan_expand_kernel(esgk::ScanArgs S) {
  using esgk::kWin;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S.nq_list) return;
  const int32_t qi = S.qlist ? S.qlist[t] : (int32_t)t;
  const int64_t a = S.l[qi], b = S.r[qi];
  const int32_t w0 = S.q_win0[qi], nwq = S.q_nwin[qi];
  for (int32_t j = 0; j < nwq; j++) {
    S.win_q[w0 + j] = qi;
    S.win_s[w0 + j] = a + (int64_t)j * kWin;
    S.win_e[w0 + j] = (a + (int64_t)(j + 1) * kWin - 1) < b ? a + (int64_t)(j + 1) * kWin - 1 : b;
  }
}

__global__ void set_i32_kernel(int32_t* p, int32_t v) { *p = v; }

void scan_expand_kernel_launch(const esgk::ScanArgs& S, hipStream_t s) {
  if (S.nq_list > 0)
    scan_expand_kernel<<<(unsigned)((S.nq_list + 255) / 256), 256, 0, s>>>(S);
}

// win_order = the windows 0..counts[0]-1 in buckets of 2^bucket_shift start
// positions, ascending (histogram, exclusive scan, scatter)
void sort_windows_by_start(esg_index* idx, int64_t nw_bound, hipStream_t s) {
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (nw_bound + 255) / 256));
  bucket_hist_kernel<<<grid, 256, 0, s>>>(idx->win_s, idx->counts, idx->bucket_shift,
                                          idx->counts + 4);
  bucket_scan_kernel<<<1, 1024, 0, s>>>(idx->counts + 4, idx->nbuckets);
  bucket_scatter_kernel<<<grid, 256, 0, s>>>(idx->win_s, idx->counts, idx->bucket_shift,
                                             idx->counts + 4, idx->win_order);
}

}  // namespace

int32_t esg_scan_batch(esg_index* idx, const esg_scan_opts* opts, const float* queries,
                       const int64_t* l, const int64_t* r, int64_t nq, int32_t k, int64_t* ids,
                       float* dists, void* stream) {
  if (!idx || nq < 0) return ESG_EINVAL;
  if (nq == 0) return ESG_OK;
  if (!queries || !l || !r || !ids || !dists || k < 1 || k > 128) return ESG_EINVAL;
  if (!idx->vec16 || !idx->norm2 || !idx->kt->scan_select[0]) return ESG_EUNSUPPORTED;
  if (idx->res_queries < 1) return ESG_ERANGE;
  if (nq > idx->res_queries) return ESG_ERANGE;
  esg_scan_opts o;
  std::memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  const int cap = 64 << scan_width_index(k);
  const int mr = o.rerank_count > 0 ? o.rerank_count : cap - 1;   // the whole list: fewest fallbacks
  if (mr < k || mr > cap - 1) return ESG_EINVAL;
  if (o.flags & ~ESG_SCAN_EXACT) return ESG_EINVAL;
  if (hipSetDevice(idx->device) != hipSuccess) return ESG_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<int64_t> hl((size_t)nq), hr((size_t)nq);
  if (hipMemcpyAsync(hl.data(), l, (size_t)nq * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(hr.data(), r, (size_t)nq * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return ESG_EHIP;
  // windows per query on the host (O(nq)); expansion and the sort by start
  // run on the device
  // a window's list takes 64E 64-bit slots of the 64 reserved per window
  const int64_t cap_windows = idx->res_windows / (1 << scan_width_index(k));
  std::vector<int32_t> q0((size_t)nq, 0), qn((size_t)nq, 0), qlist;
  int64_t n_fallback = 0;
  int64_t qa = 0;
  while (qa < nq) {
    // one pass: queries [qa, qb) whose windows fit the reservation
    int64_t qb = qa, nw = 0;
    qlist.clear();
    for (; qb < nq; qb++) {
      const int64_t a = hl[(size_t)qb], b = hr[(size_t)qb];
      const bool valid = a >= 0 && b < idx->n && a <= b;
      const int64_t nwq = valid ? (b - a + esgk::kWin) / esgk::kWin : 0;
      if (nw + nwq > cap_windows && qb > qa) break;
      if (nwq > cap_windows) return ESG_ERANGE;
      q0[(size_t)qb] = (int32_t)nw;
      qn[(size_t)qb] = (int32_t)nwq;
      nw += nwq;
      qlist.push_back((int32_t)qb);
    }
    bool ok = hipMemcpyAsync(idx->q_win0, q0.data(), (size_t)nq * 4, hipMemcpyHostToDevice, s) ==
                  hipSuccess &&
              hipMemcpyAsync(idx->q_nwin, qn.data(), (size_t)nq * 4, hipMemcpyHostToDevice, s) ==
                  hipSuccess &&
              hipMemcpyAsync(idx->qlist, qlist.data(), qlist.size() * 4, hipMemcpyHostToDevice,
                             s) == hipSuccess;
    if (!ok) return ESG_EHIP;
    esgk::ScanArgs S = scan_args(idx, queries, l, r, nq, k, mr, ids, dists, o.certified);
    S.force_exact = (o.flags & ESG_SCAN_EXACT) ? 1 : 0;
    S.qlist = idx->qlist;
    S.nw = nw;
    S.nq_list = (int64_t)qlist.size();
    S.win_order = idx->win_order;
    zero_i32_kernel<<<1, 1024, 0, s>>>(idx->counts, 4 + idx->nbuckets);
    set_i32_kernel<<<1, 1, 0, s>>>(idx->counts, (int32_t)nw);
    scan_expand_kernel_launch(S, s);
    sort_windows_by_start(idx, nw, s);
    S.n_win_dev = nullptr;
    int32_t st = launch_scan(idx, S, nw, (int64_t)qlist.size(), s);
    if (st != ESG_OK) return st;
    int32_t nfb = 0;
    if (hipMemcpyAsync(&nfb, idx->counts + 2, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return ESG_EHIP;
    n_fallback += nfb;
    qa = qb;
  }
  if (o.n_fallback) *o.n_fallback = n_fallback;
  return ESG_OK;
}

namespace {

int32_t launch_search(esg_index* idx, const esgk::SearchArgs& a0, const void* fn, size_t lds,
                      int64_t nq_bound, hipStream_t s) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * esgk::kWavesPerGroup, lds) !=
      hipSuccess) {
    (void)hipGetLastError();
    return ESG_EHIP;
  }
  if (per_cu < 1) return ESG_ERANGE;  // the LDS request does not fit one CU
  int64_t grid = std::min<int64_t>((nq_bound + esgk::kWavesPerGroup - 1) / esgk::kWavesPerGroup,
                                   (int64_t)per_cu * idx->cu_count);
  grid = std::min<int64_t>(grid, idx->spill_slots / esgk::kWavesPerGroup);
  reset_counter_kernel<<<1, 1, 0, s>>>(idx->counter);
  esgk::SearchArgs a = a0;
  void* args[] = {&a};
  if (hipLaunchKernel(fn, dim3((unsigned)grid), dim3(64 * esgk::kWavesPerGroup), args, lds, s) !=
      hipSuccess) {
    (void)hipGetLastError();
    return ESG_EHIP;
  }
  return ESG_OK;
}

// Router: narrow queries take the scan, the rest the graph search.  Every
// size the host needs is an upper bound (nq), so the sequence can be
// captured in a graph; the kernels read the actual counts on the device.
int32_t launch_routed(esg_index* idx, const esgk::SearchArgs& a, const void* fn, size_t lds,
                      int64_t thr, int32_t mr, hipStream_t s) {
  const int64_t nq = a.nq;
  zero_i32_kernel<<<1, 1024, 0, s>>>(idx->counts, 4 + idx->nbuckets);
  classify_kernel<<<(unsigned)((nq + 255) / 256), 256, 0, s>>>(
      a.l, a.r, nq, idx->n, thr, idx->win_q, idx->win_s, idx->win_e, idx->q_win0, idx->q_nwin,
      idx->wide, idx->counts);
  const unsigned sgrid = (unsigned)std::min<int64_t>(1024, (nq + 255) / 256);
  bucket_hist_kernel<<<sgrid, 256, 0, s>>>(idx->win_s, idx->counts, idx->bucket_shift,
                                           idx->counts + 4);
  bucket_scan_kernel<<<1, 1024, 0, s>>>(idx->counts + 4, idx->nbuckets);
  bucket_scatter_kernel<<<sgrid, 256, 0, s>>>(idx->win_s, idx->counts, idx->bucket_shift,
                                              idx->counts + 4, idx->win_order);
  esgk::ScanArgs S = scan_args(idx, a.queries, a.l, a.r, nq, a.k, mr, a.ids, a.dists, nullptr);
  S.qlist = idx->win_q;          // narrow window i belongs to query win_q[i]
  S.n_win_dev = idx->counts;
  S.n_q_dev = idx->counts;
  S.nw = nq;
  S.nq_list = nq;
  int32_t st = launch_scan(idx, S, nq, nq, s);
  if (st != ESG_OK) return st;
  esgk::SearchArgs w = a;
  w.qlist = idx->wide;
  w.qcount = idx->counts + 1;
  return launch_search(idx, w, fn, lds, nq, s);
}

}  // namespace

int32_t esg_search_batch_ex(esg_index* idx, const esg_search_opts* opts, const float* queries,
                            const int64_t* l, const int64_t* r, int64_t nq, int32_t k, int32_t ef,
                            int64_t* ids, float* dists, void* stream) {
  if (!idx || nq < 0) return ESG_EINVAL;
  if (nq == 0) return ESG_OK;
  if (!queries || !l || !r || !ids || !dists) return ESG_EINVAL;
  if (k < 1 || ef < k || ef > ESG_EF_MAX) return ESG_EINVAL;
  if (nq > 0x7FFFFFFFll) return ESG_ERANGE;
  esg_search_opts o;
  std::memset(&o, 0, sizeof(o));
  o.hop_budget = -1;
  if (opts) o = *opts;
  const int cand_cap = o.cand_cap == 0 ? ef : o.cand_cap;
  if (cand_cap < 1 || cand_cap > ESG_EF_MAX) return ESG_EINVAL;
  const int hash_cap = o.hash_cap == 0 ? kDefaultHashCap : o.hash_cap;
  if (hash_cap < 64 || hash_cap > 16384 || (hash_cap & (hash_cap - 1)) != 0) return ESG_EINVAL;
  // a slot stores the low kb - log2(hash_cap) <= 12 bits of a node-local key
  int tbits = 0;
  while ((1 << tbits) < hash_cap) tbits++;
  int kb = 0;
  while (kb < 32 && ((int64_t)1 << kb) < idx->n) kb++;
  if (kb - tbits > 12) return ESG_ERANGE;
  if (o.traversal < ESG_TRAV_F32 || o.traversal > ESG_TRAV_FP8) return ESG_EINVAL;
  if (o.traversal == ESG_TRAV_BF16 && !idx->vec16) return ESG_EUNSUPPORTED;
  if (o.traversal == ESG_TRAV_FP8 && !idx->vec8) return ESG_EUNSUPPORTED;
  if ((o.trace || o.visited) && nq > ((int64_t)1 << 40)) return ESG_ERANGE;
  if (o.visited && o.visited_cap < 1) return ESG_EINVAL;
  int32_t mr = 0;
  if (o.router_threshold > 0) {
    if (!idx->vec16 || !idx->norm2 || !idx->kt->scan_select[0]) return ESG_EUNSUPPORTED;
    if (k > 128) return ESG_EINVAL;
    if (nq > idx->res_queries || nq > idx->res_windows / (1 << scan_width_index(k)))
      return ESG_ERANGE;
    if (o.router_threshold > esgk::kWin) return ESG_EINVAL;
    const int cap = 64 << scan_width_index(k);
    mr = o.scan_rerank > 0 ? o.scan_rerank : cap - 1;
    if (mr < k || mr > cap - 1) return ESG_EINVAL;
  }

  // kernel: plain, or with the learned switch after a one-hop or a longer probe
  // probe_hops = 0 with a network (or feat_out): beams chosen before the
  // search by predict_beams_kernel, then the plain kernel
  const bool predict = (o.mlp || o.feat_out) && o.probe_hops == 0;
  const int learn = ((o.mlp || o.feat_out) && o.probe_hops > 0) ? (o.probe_hops == 1 ? 1 : 2) : 0;
  const void* fn = idx->kt->fn[o.traversal][width_index(std::max(ef, cand_cap))][learn];
  if (!fn) return ESG_EUNSUPPORTED;

  esgk::SearchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.vec = idx->vec;
  a.vec16 = idx->vec16;
  a.vec8 = idx->vec8;
  a.scale8 = idx->scale8;
  a.adj = idx->adj;
  a.ep = idx->ep;
  a.ext_id = idx->ext_id;
  a.n = idx->n;
  a.d = idx->d;
  a.dq = idx->dq;
  a.dp = idx->dp;
  a.R = idx->R;
  a.leaf = idx->leaf;
  a.n_depth = idx->n_depth;
  a.c_den = idx->c_den;
  a.fanout = idx->fanout;
  a.layout = idx->layout;
  a.row_base = idx->row_base;
  a.queries = queries;
  a.l = l;
  a.r = r;
  a.nq = nq;
  a.k = k;
  a.ef = ef;
  a.cand_cap = cand_cap;
  a.rerank = o.rerank;
  a.hop_budget = o.hop_budget;
  a.ids = ids;
  a.dists = dists;
  a.trace = o.trace;
  a.visited = o.visited;
  a.visited_cap = o.visited ? o.visited_cap : 0;
  a.n_invalid = o.n_invalid;
  a.spill = idx->spill;
  a.spill_words = idx->spill_words;
  a.spill_slots = idx->spill_slots;
  a.counter = idx->counter;
  a.hash_cap = hash_cap;
  if (o.probe_hops < 0) return ESG_EINVAL;
  a.mlp = o.mlp ? idx->mlp_pack : nullptr;
  a.feat_out = o.feat_out;
  a.probe_hops = (o.mlp || o.feat_out) ? o.probe_hops : 0;
  a.mlp_delta = o.mlp_delta;
  if (o.mlp_target < 0 || o.mlp_target > 1) return ESG_EINVAL;
  a.mlp_target = o.mlp_target;
  if (o.part_ef) {
    if (o.mlp) return ESG_EINVAL;
    a.part_ef = o.part_ef;
  }
  esgk::SearchArgs pa = a;   // the predictor's arguments
  if (predict) {
    if (o.mlp_target != 0) return ESG_EINVAL;   // a stopping step needs a probe
    if (nq > idx->res_queries) return ESG_ERANGE;
    pa.feat_out = o.feat_out;
    a.mlp = nullptr;
    a.feat_out = nullptr;
    a.probe_hops = 0;
    if (o.mlp) a.part_ef = idx->part_ef;
  }

  if (hipSetDevice(idx->device) != hipSuccess) return ESG_EHIP;
  const size_t lds = (size_t)esgk::kWavesPerGroup * (esgk::kStageBytes + 2 * (size_t)hash_cap);
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto sequence = [&](hipStream_t st) -> int32_t {
    if (o.mlp && !predict) {
      mlp_pack_kernel<<<(esgk::kMlpParams + 255) / 256, 256, 0, st>>>(o.mlp, idx->mlp_pack);
      if (hipGetLastError() != hipSuccess) return ESG_EHIP;
    }
    if (predict && nq > 0) {
      predict_beams_kernel<<<(unsigned)((nq + 255) / 256), 256, 0, st>>>(pa, o.mlp,
                                                                        idx->part_ef);
      if (hipGetLastError() != hipSuccess) return ESG_EHIP;
    }
    return o.router_threshold > 0 ? launch_routed(idx, a, fn, lds, o.router_threshold, mr, st)
                                  : launch_search(idx, a, fn, lds, nq, st);
  };
  if (!o.use_graph) return sequence(s);

  // hipGraph: capture once per argument set on the library's own stream,
  // replay on the caller's stream.
  if (!idx->capture_stream &&
      hipStreamCreateWithFlags(&idx->capture_stream, hipStreamNonBlocking) != hipSuccess)
    return ESG_EHIP;
  std::vector<uint8_t> key(sizeof(a) + sizeof(o) + 8);
  std::memcpy(key.data(), &a, sizeof(a));
  std::memcpy(key.data() + sizeof(a), &o, sizeof(o));
  std::memcpy(key.data() + sizeof(a) + sizeof(o), &mr, 4);
  hipGraphExec_t exec = nullptr;
  for (auto& g : idx->graphs)
    if (g.key == key) exec = g.exec;
  if (!exec) {
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(idx->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return ESG_EHIP;
    const int32_t st = sequence(idx->capture_stream);
    const hipError_t e = hipStreamEndCapture(idx->capture_stream, &graph);
    if (st != ESG_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return st != ESG_OK ? st : ESG_EHIP;
    }
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      (void)hipGetLastError();
      return ESG_EHIP;
    }
    if (idx->graphs.size() >= 16) {
      (void)hipGraphExecDestroy(idx->graphs.front().exec);
      idx->graphs.erase(idx->graphs.begin());
    }
    idx->graphs.push_back({key, exec});
  }
  if (hipGraphLaunch(exec, s) != hipSuccess) {
    (void)hipGetLastError();
    return ESG_EHIP;
  }
  return ESG_OK;
}

int32_t esg_search_batch(esg_index* idx, const float* queries, const int64_t* l, const int64_t* r,
                         int64_t nq, int32_t k, int32_t ef, int64_t* ids, float* dists,
                         void* stream) {
  return esg_search_batch_ex(idx, nullptr, queries, l, r, nq, k, ef, ids, dists, stream);
}

}  // extern "C"

// ---- device side of the index builder --------------------------------------------------

namespace {

__global__ void identity_kernel(int64_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = i;
}

// Query rows of the round: the inserted points' own vectors.
__global__ void build_gather_kernel(const float* __restrict__ vec, int64_t dp, int32_t d,
                                    const uint32_t* __restrict__ pts, int64_t nb,
                                    float* __restrict__ q) {
  const int64_t total = nb * d;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / d, j = i % d;
    q[i] = vec[(int64_t)pts[b] * dp + j];
  }
}

// Reverse-edge proposals (target c <- source p) grouped by target without a
// sort: count per target (the first proposal registers the target), give
// each target a segment, then fill the segments.  Segment layout and the
// order inside a segment depend on atomic order; the consumer sorts what
// it uses, so the rows written do not.
__global__ void build_count_kernel(const uint32_t* __restrict__ pts, int64_t nb,
                                   const uint32_t* __restrict__ rows, int32_t R,
                                   int32_t* __restrict__ cnt, int32_t* __restrict__ touched,
                                   int32_t* __restrict__ counters) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb * R) return;
  const uint32_t c = rows[(int64_t)pts[i / R] * R + i % R];
  if (c == ESG_NO_NODE) return;
  if (atomicAdd(&cnt[c], 1) == 0) touched[atomicAdd(&counters[0], 1)] = (int32_t)c;
}

__global__ void build_alloc_kernel(const int32_t* __restrict__ touched,
                                   const int32_t* __restrict__ cnt, int32_t* __restrict__ start,
                                   int32_t* __restrict__ fill, int32_t* __restrict__ counters,
                                   int64_t bound) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= bound || u >= counters[0]) return;
  const int32_t c = touched[u];
  start[c] = atomicAdd(&counters[1], cnt[c]);
  fill[c] = 0;
}

__global__ void build_fill_kernel(const uint32_t* __restrict__ pts, int64_t nb,
                                  const uint32_t* __restrict__ rows, int32_t R,
                                  const int32_t* __restrict__ start, int32_t* __restrict__ fill,
                                  uint32_t* __restrict__ srcs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb * R) return;
  const uint32_t p = pts[i / R];
  const uint32_t c = rows[(int64_t)p * R + i % R];
  if (c == ESG_NO_NODE) return;
  srcs[start[c] + atomicAdd(&fill[c], 1)] = p;
}

__global__ void build_reset_kernel(int32_t* counters) {
  counters[0] = 0;
  counters[1] = 0;
}

}  // namespace

namespace esgb {

struct GpuState {
  esg_index ix;                 // vectors, adjacency of every depth, search workspace
  int32_t efc = 0, hash_cap = 0, max_lds = 0;
  int64_t max_round = 0;
  uint32_t* pts = nullptr;      // [max_round] round arrays
  uint32_t* eps = nullptr;
  int64_t* l = nullptr;
  int64_t* r = nullptr;
  float* qbuf = nullptr;        // [max_round][d]
  int64_t* cid = nullptr;       // [max_round][efc]
  float* cd = nullptr;
  int32_t* cnt = nullptr;       // [n]
  int32_t* start = nullptr;
  int32_t* fill = nullptr;
  int32_t* touched = nullptr;   // [max_round * R]
  uint32_t* srcs = nullptr;
  int32_t* counters = nullptr;  // [0] touched targets, [1] proposals placed
  std::vector<uint32_t> h32;    // host staging
  std::vector<int64_t> h64;
};

int32_t gpu_open(int32_t device, const float* X, int64_t n, int32_t d, int32_t R,
                 int32_t n_depth, int32_t efc, int64_t max_round, GpuState** out) {
  if (!out || !X || n < 1 || n >= (int64_t)ESG_NO_NODE || d < 1 || d > 65536 || R < 1 ||
      R > ESG_DEGREE_MAX || n_depth < 1 || n_depth > 40 || efc < 1 || max_round < 1)
    return ESG_EINVAL;
  if (efc > ESG_EF_MAX) return ESG_EUNSUPPORTED;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) {
    (void)hipGetLastError();
    return ESG_EHIP;
  }
  if (device < 0 || device >= ndev) return ESG_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return ESG_EHIP;
  const esgk::KernelTable* kt = nullptr;
  for (const auto& t : kernel_tables())
    if (!kt && same_shape(d, t.dim)) kt = &t;
  if (!kt || !kt->build_prune || !kt->build_search[width_index(efc)]) return ESG_EUNSUPPORTED;
  // the visited hash keeps the low bits of a node-local key: <= 12 spare bits
  int kb = 0;
  while (kb < 32 && ((int64_t)1 << kb) < n) kb++;
  int hash_cap = kDefaultHashCap;
  while (hash_cap < 16384 && kb - __builtin_ctz((unsigned)hash_cap) > 12) hash_cap *= 2;
  if (kb - __builtin_ctz((unsigned)hash_cap) > 12) return ESG_ERANGE;

  GpuState* g = new (std::nothrow) GpuState();
  if (!g) return ESG_ENOMEM;
  esg_index& ix = g->ix;
  ix.device = device;
  ix.n = n;
  ix.d = d;
  ix.dq = d;
  ix.dp = (d + 15) / 16 * 16;
  ix.R = R;
  ix.leaf = 1;
  ix.n_depth = n_depth;
  ix.kt = kt;
  g->efc = efc;
  g->hash_cap = hash_cap;
  g->max_round = max_round;
  if (hipDeviceGetAttribute(&ix.cu_count, hipDeviceAttributeMultiprocessorCount, device) !=
          hipSuccess ||
      hipDeviceGetAttribute(&g->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
          hipSuccess) {
    delete g;
    return ESG_EHIP;
  }
  ix.spill_slots = (int64_t)ix.cu_count * 32;
  ix.spill_words = ((n + 31) / 32 + 63) / 64 * 64;
  int32_t st = ESG_OK;
  auto A = [&](void** p, size_t b) {
    if (st == ESG_OK) st = ix.alloc(p, b);
  };
  const size_t spill_bytes = (size_t)ix.spill_slots * (ix.spill_words + esgk::kSpillLog) * 4;
  const size_t M = (size_t)max_round;
  A((void**)&ix.vec, (size_t)n * ix.dp * 4);
  A((void**)&ix.adj, (size_t)n_depth * n * R * 4);
  A((void**)&ix.ext_id, (size_t)n * 8);
  A((void**)&ix.spill, spill_bytes);
  A((void**)&ix.counter, 256);
  A((void**)&ix.row_base, (size_t)n_depth * 8);
  A((void**)&g->pts, M * 4);
  A((void**)&g->eps, M * 4);
  A((void**)&g->l, M * 8);
  A((void**)&g->r, M * 8);
  A((void**)&g->qbuf, M * d * 4);
  A((void**)&g->cid, M * efc * 8);
  A((void**)&g->cd, M * efc * 4);
  A((void**)&g->cnt, (size_t)n * 4);
  A((void**)&g->start, (size_t)n * 4);
  A((void**)&g->fill, (size_t)n * 4);
  A((void**)&g->touched, M * R * 4);
  A((void**)&g->srcs, M * R * 4);
  A((void**)&g->counters, 8);
  if (st != ESG_OK) {
    ix.release();
    delete g;
    return st;
  }
  std::vector<int64_t> rb((size_t)n_depth);
  for (int t = 0; t < n_depth; t++) rb[(size_t)t] = (int64_t)t * n;
  identity_kernel<<<1024, 256>>>(ix.ext_id, n);
  const bool ok = hipGetLastError() == hipSuccess &&
                  hipMemcpy(ix.row_base, rb.data(), rb.size() * 8, hipMemcpyHostToDevice) ==
                      hipSuccess &&
                  hipMemset(ix.counter, 0, 256) == hipSuccess &&
                  hipMemset(ix.spill, 0, spill_bytes) == hipSuccess &&
                  hipMemset(g->cnt, 0, (size_t)n * 4) == hipSuccess &&
                  hipDeviceSynchronize() == hipSuccess;
  if (!ok || (st = gpu_reset(g, X)) != ESG_OK) {
    (void)hipGetLastError();
    ix.release();
    delete g;
    return st != ESG_OK ? st : ESG_EHIP;
  }
  *out = g;
  return ESG_OK;
}

int32_t gpu_reset(GpuState* g, const float* X) {
  if (!g || !X) return ESG_EINVAL;
  esg_index& ix = g->ix;
  if (hipSetDevice(ix.device) != hipSuccess) return ESG_EHIP;
  const bool ok =
      hipDeviceSynchronize() == hipSuccess &&
      h2d_rows(ix.vec, (size_t)ix.dp * 4, X, (size_t)ix.d * 4, (size_t)ix.d * 4, (size_t)ix.n) &&
      hipMemset(ix.adj, 0xFF, (size_t)ix.n_depth * ix.n * ix.R * 4) == hipSuccess &&   // ESG_NO_NODE
      hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    return ESG_EHIP;
  }
  // the rows on the device are checked against X (as the loader checks its copy)
  const int v = verify_upload(ix.vec, X, ix.n, ix.d, ix.dp);
  if (v != 1) {
    if (v == 0) std::fprintf(stderr, "esg builder: the device copy of the vectors differs\n");
    return ESG_EHIP;
  }
  return ESG_OK;
}

int32_t gpu_copy_rows(GpuState* g, int32_t dst, int32_t src, int64_t a, int64_t count) {
  if (!g) return ESG_EINVAL;
  esg_index& ix = g->ix;
  if (dst < 0 || src < 0 || dst >= ix.n_depth || src >= ix.n_depth || a < 0 || count < 0 ||
      a + count > ix.n)
    return ESG_EINVAL;
  if (hipSetDevice(ix.device) != hipSuccess) return ESG_EHIP;
  const size_t row = (size_t)ix.R;
  if (hipMemcpy(ix.adj + ((size_t)dst * ix.n + a) * row, ix.adj + ((size_t)src * ix.n + a) * row,
                (size_t)count * row * 4, hipMemcpyDeviceToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return ESG_EHIP;
  }
  return ESG_OK;
}

int32_t gpu_get_rows(GpuState* g, int32_t depth, uint32_t* rows) {
  if (!g || !rows || depth < 0 || depth >= g->ix.n_depth) return ESG_EINVAL;
  esg_index& ix = g->ix;
  if (hipSetDevice(ix.device) != hipSuccess) return ESG_EHIP;
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(rows, ix.adj + (size_t)depth * ix.n * ix.R, (size_t)ix.n * ix.R * 4,
                hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return ESG_EHIP;
  }
  return ESG_OK;
}

int32_t gpu_put_rows(GpuState* g, int32_t depth, const uint32_t* rows) {
  if (!g || !rows || depth < 0 || depth >= g->ix.n_depth) return ESG_EINVAL;
  esg_index& ix = g->ix;
  if (hipSetDevice(ix.device) != hipSuccess) return ESG_EHIP;
  if (!h2d(ix.adj + (size_t)depth * ix.n * ix.R, rows, (size_t)ix.n * ix.R * 4) ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    return ESG_EHIP;
  }
  return ESG_OK;
}

namespace {

// One chunk of a round (whole jobs, at most max_round points).
int32_t round_chunk(GpuState* g, int32_t depth, int64_t nb, const uint32_t* pts,
                    const uint32_t* eps, const uint32_t* lo, const uint32_t* hi,
                    int32_t max_batch) {
  esg_index& ix = g->ix;
  const int R = ix.R, efc = g->efc;
  // host staging: positions, entries, ranges [lo, hi] of the current graphs
  g->h64.resize((size_t)nb * 2);
  for (int64_t i = 0; i < nb; i++) {
    g->h64[(size_t)i] = lo[i];
    g->h64[(size_t)(nb + i)] = hi[i];
  }
  if (hipDeviceSynchronize() != hipSuccess ||   // the previous round has read these buffers
      hipMemcpy(g->pts, pts, (size_t)nb * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(g->eps, eps, (size_t)nb * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(g->l, g->h64.data(), (size_t)nb * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(g->r, g->h64.data() + nb, (size_t)nb * 8, hipMemcpyHostToDevice) != hipSuccess)
    return ESG_EHIP;
  const unsigned gblocks = (unsigned)std::min<int64_t>(4096, (nb * ix.d + 255) / 256);
  build_gather_kernel<<<gblocks, 256>>>(ix.vec, ix.dp, ix.d, g->pts, nb, g->qbuf);

  // 1) insertion searches: Alg. 1 from each point's entry on its graph's
  //    positions, beam width = candidates kept = efc
  esgk::SearchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.vec = ix.vec;
  a.adj = ix.adj;
  a.ep = g->eps;
  a.ext_id = ix.ext_id;
  a.n = ix.n;
  a.d = ix.d;
  a.dq = ix.d;
  a.dp = ix.dp;
  a.R = R;
  a.leaf = 1;
  a.n_depth = ix.n_depth;
  a.c_den = 2;
  a.fanout = 2;
  a.row_base = ix.row_base;
  a.forced_depth = depth;
  a.queries = g->qbuf;
  a.l = g->l;
  a.r = g->r;
  a.nq = nb;
  a.k = efc;
  a.ef = efc;
  a.cand_cap = efc;
  a.hop_budget = -1;
  a.ids = g->cid;
  a.dists = g->cd;
  a.spill = ix.spill;
  a.spill_words = ix.spill_words;
  a.spill_slots = ix.spill_slots;
  a.counter = ix.counter;
  a.hash_cap = g->hash_cap;
  const void* fn = ix.kt->build_search[width_index(efc)];
  const size_t slds = (size_t)esgk::kWavesPerGroup * (esgk::kStageBytes + 2 * (size_t)g->hash_cap);
  int32_t st = launch_search(&ix, a, fn, slds, nb, nullptr);
  if (st != ESG_OK) return st;

  // 2) forward rows, 3) reverse edges
  int keycap = 1;
  while (keycap < std::max(efc, R + max_batch)) keycap <<= 1;
  esgk::BuildArgs B;
  std::memset(&B, 0, sizeof(B));
  B.A = a;
  B.nb = nb;
  B.efc = efc;
  B.R = R;
  B.keycap = keycap;
  B.wave_lds = esgk::kStageBytes + keycap * 8 + 32 * 4;
  B.pts = g->pts;
  B.cand_ids = g->cid;
  B.cand_d = g->cd;
  B.rows = ix.adj + (size_t)depth * ix.n * R;
  B.cnt = g->cnt;
  B.start = g->start;
  B.srcs = g->srcs;
  B.touched = g->touched;
  B.counters = g->counters;
  const int wpb = std::max(1, std::min(esgk::kWavesPerGroup, g->max_lds / B.wave_lds));
  if (B.wave_lds > g->max_lds) return ESG_EUNSUPPORTED;
  const size_t blds = (size_t)wpb * B.wave_lds;
  void* args[] = {&B};
  if (hipLaunchKernel(ix.kt->build_prune, dim3((unsigned)((nb + wpb - 1) / wpb)), dim3(64 * wpb),
                      args, blds, nullptr) != hipSuccess)
    return ESG_EHIP;
  const int64_t np = nb * R;
  const unsigned pblocks = (unsigned)((np + 255) / 256);
  build_reset_kernel<<<1, 1>>>(g->counters);
  build_count_kernel<<<pblocks, 256>>>(g->pts, nb, B.rows, R, g->cnt, g->touched, g->counters);
  build_alloc_kernel<<<pblocks, 256>>>(g->touched, g->cnt, g->start, g->fill, g->counters, np);
  build_fill_kernel<<<pblocks, 256>>>(g->pts, nb, B.rows, R, g->start, g->fill, g->srcs);
  const unsigned rblocks =
      (unsigned)std::min<int64_t>((np + wpb - 1) / wpb, (int64_t)ix.cu_count * 16);
  if (hipLaunchKernel(ix.kt->build_reverse, dim3(rblocks), dim3(64 * wpb), args, blds, nullptr) !=
      hipSuccess)
    return ESG_EHIP;
  return hipGetLastError() == hipSuccess ? ESG_OK : ESG_EHIP;
}

}  // namespace

int32_t gpu_round(GpuState* g, int32_t depth, int64_t nb, const uint32_t* pts,
                  const uint32_t* eps, const uint32_t* lo, const uint32_t* hi) {
  if (!g || depth < 0 || depth >= g->ix.n_depth || nb < 0 || (nb > 0 && (!pts || !eps || !lo || !hi)))
    return ESG_EINVAL;
  esg_index& ix = g->ix;
  for (int64_t i = 0; i < nb; i++)
    if (pts[i] >= ix.n || eps[i] >= ix.n || lo[i] > hi[i] || hi[i] >= ix.n || pts[i] <= hi[i] ||
        eps[i] < lo[i] || eps[i] > hi[i])
      return ESG_EINVAL;
  if (hipSetDevice(ix.device) != hipSuccess) return ESG_EHIP;
  // chunks of whole jobs (a job's points are consecutive and share lo)
  int64_t i0 = 0;
  while (i0 < nb) {
    int64_t i1 = i0, max_batch = 0;
    while (i1 < nb) {
      int64_t j = i1;
      while (j < nb && lo[j] == lo[i1]) j++;
      if (j - i0 > g->max_round && i1 > i0) break;
      if (j - i1 > g->max_round) return ESG_EINVAL;   // one job's batch exceeds a round
      max_batch = std::max(max_batch, j - i1);
      i1 = j;
    }
    const int32_t st =
        round_chunk(g, depth, i1 - i0, pts + i0, eps + i0, lo + i0, hi + i0, (int32_t)max_batch);
    if (st != ESG_OK) {
      (void)hipGetLastError();
      return st;
    }
    i0 = i1;
  }
  return ESG_OK;
}

void gpu_close(GpuState* g) {
  if (!g) return;
  if (hipSetDevice(g->ix.device) == hipSuccess) (void)hipDeviceSynchronize();
  g->ix.release();
  delete g;
}

}  // namespace esgb
