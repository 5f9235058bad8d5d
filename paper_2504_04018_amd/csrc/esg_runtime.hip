// libesg host runtime: index loading, storage codecs, launch of the search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/esg.h"
#include "esg_dims.h"
#include "esg_dispatch.h"
#include "esg_format.h"
#include "esg_kernels.h"

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
  int32_t d = 0, dp = 0, R = 0, leaf = 0, n_depth = 0, c_den = 2;
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
    for (void* p : allocations) (void)hipFree(p);
    allocations.clear();
  }
};

namespace {

__global__ void reset_counter_kernel(uint32_t* c) { *c = 0u; }

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

bool tree_is_consistent(int64_t n, int32_t leaf, int32_t n_depth, int32_t R, const uint32_t* adj,
                        const uint32_t* ep) {
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
    const int64_t mid = (nd.a + nd.b) / 2;
    todo.push_back({nd.a, mid, 2 * nd.heap, nd.depth + 1});
    todo.push_back({mid + 1, nd.b, 2 * nd.heap + 1, nd.depth + 1});
  }
  return true;
}

int width_index(int cap) {
  if (cap <= 64) return 0;
  if (cap <= 128) return 1;
  if (cap <= 256) return 2;
  if (cap <= 512) return 3;
  return 4;
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
      h.degree > ESG_DEGREE_MAX || h.leaf < 1 || h.fanout != 2 || h.n_depth < 0 ||
      h.n_depth > 40 || h.c_den < 1)
    return ESG_EFORMAT;
  const uint64_t sizes[5] = {esg::bytes_ids(h.n), esg::bytes_attr(h.n), esg::bytes_vec(h.n, h.d),
                             esg::bytes_adj(h.n, h.n_depth, h.degree), esg::bytes_ep(h.n_depth)};
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
    if (t.dim == h.d) kt = &t;
  if (!kt) return ESG_EUNSUPPORTED;

  std::vector<int64_t> ids((size_t)h.n);
  std::vector<float> vec((size_t)h.n * (size_t)h.d);
  std::vector<uint32_t> adj((size_t)h.n_depth * (size_t)h.n * (size_t)h.degree);
  std::vector<uint32_t> ep((size_t)1 << h.n_depth);
  std::vector<double> attr((size_t)h.n);
  void* dsts[5] = {ids.data(), attr.data(), vec.data(), adj.data(), ep.data()};
  for (int s = 0; s < 5; s++) {
    if (!read_exact(f, offs[s], dsts[s], sizes[s])) return ESG_EIO;
    if (crc.update(0, dsts[s], sizes[s]) != h.crc_sections[s]) return ESG_EFORMAT;
  }
  // Structural checks the kernels rely on: every graph node [a,b] of the
  // tree has its entry point and all neighbours of its rows inside [a,b].
  if (!tree_is_consistent(h.n, h.leaf, h.n_depth, h.degree, adj.data(), ep.data()))
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
  A((void**)&ix->spill, (size_t)ix->spill_slots * ix->spill_words * 4);
  A((void**)&ix->counter, 256);
  if (st != ESG_OK) {
    ix->release();
    delete ix;
    return st;
  }
  bool ok = hipMemset(ix->vec, 0, (size_t)h.n * ix->dp * 4) == hipSuccess &&
            hipMemcpy2D(ix->vec, (size_t)ix->dp * 4, vec.data(), (size_t)h.d * 4, (size_t)h.d * 4,
                        (size_t)h.n, hipMemcpyHostToDevice) == hipSuccess &&
            (adj.empty() ||
             hipMemcpy(ix->adj, adj.data(), adj.size() * 4, hipMemcpyHostToDevice) == hipSuccess) &&
            hipMemcpy(ix->ep, ep.data(), ep.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(ix->ext_id, ids.data(), ids.size() * 8, hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemset(ix->counter, 0, 256) == hipSuccess &&
            hipDeviceSynchronize() == hipSuccess;
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
  out->fanout = 2;
  out->n_depth = idx->n_depth;
  out->c_den = idx->c_den;
  out->has_bf16 = idx->vec16 != nullptr;
  out->has_fp8 = idx->vec8 != nullptr;
  out->device_bytes = idx->device_bytes;
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
    if (st != ESG_OK) return st;
    encode_bf16_kernel<<<4096, 256, 0, s>>>(idx->vec, idx->vec16, count);
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

  const void* fn = idx->kt->fn[o.traversal][width_index(std::max(ef, cand_cap))];
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
  a.dp = idx->dp;
  a.R = idx->R;
  a.leaf = idx->leaf;
  a.n_depth = idx->n_depth;
  a.c_den = idx->c_den;
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

  if (hipSetDevice(idx->device) != hipSuccess) return ESG_EHIP;
  const size_t lds = (size_t)esgk::kWavesPerGroup * (esgk::kStageBytes + 2 * (size_t)hash_cap);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * esgk::kWavesPerGroup, lds) !=
      hipSuccess) {
    (void)hipGetLastError();
    return ESG_EHIP;
  }
  if (per_cu < 1) return ESG_ERANGE;  // the LDS request does not fit one CU
  int64_t grid = std::min<int64_t>((nq + esgk::kWavesPerGroup - 1) / esgk::kWavesPerGroup,
                                   (int64_t)per_cu * idx->cu_count);
  grid = std::min<int64_t>(grid, idx->spill_slots / esgk::kWavesPerGroup);
  hipStream_t s = static_cast<hipStream_t>(stream);
  reset_counter_kernel<<<1, 1, 0, s>>>(idx->counter);
  void* args[] = {&a};
  if (hipLaunchKernel(fn, dim3((unsigned)grid), dim3(64 * esgk::kWavesPerGroup), args, lds, s) !=
      hipSuccess) {
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
