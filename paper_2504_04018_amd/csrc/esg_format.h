// Index file layout shared by the host builder and the loader of libesg.
// The byte layout is documented in include/esg.h (index file, version 1).
#pragma once

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <vector>

namespace esg {

constexpr char kMagic[8] = {'E', 'S', 'G', 'I', 'D', 'X', '0', '1'};
constexpr uint32_t kVersion = 2;
constexpr uint32_t kHeaderBytes = 512;
constexpr uint64_t kAlign = 4096;

#pragma pack(push, 1)
struct FileHeader {
  char magic[8];
  uint32_t version;
  uint32_t header_bytes;
  int64_t n;
  int32_t d, degree, leaf, fanout, n_depth, c_den, ef_construction, layout;
  uint64_t off_ids, off_attr, off_vec, off_adj, off_ep, file_bytes;
  uint32_t crc_sections[5];
  int32_t metric;      // ESG_METRIC_*: what the stored vectors were made from
  int32_t dq;          // query length: d, or d - 1 for the inner-product transform
  double max_norm2;    // inner product: M^2, the largest squared norm; else 0
  uint32_t crc_header; // crc32c of bytes [0, offsetof(crc_header))
};
#pragma pack(pop)
static_assert(sizeof(FileHeader) == 144, "header layout");
static_assert(offsetof(FileHeader, crc_header) == 140, "header layout");

inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Section sizes in bytes.
inline uint64_t bytes_ids(int64_t n) { return (uint64_t)n * 8; }
inline uint64_t bytes_attr(int64_t n) { return (uint64_t)n * 8; }
inline uint64_t bytes_vec(int64_t n, int32_t d) { return (uint64_t)n * (uint64_t)d * 4; }
inline uint64_t bytes_adj(int64_t n, int32_t depth, int32_t r) {
  return (uint64_t)depth * (uint64_t)n * (uint64_t)r * 4;
}
// Entry-point table: tree nodes are numbered breadth-first from the root 1
// (child j of node h is fanout*(h-1) + 2 + j), so the nodes of depths
// 0..depth-1 take the numbers 1 .. sum of fanout^t; slot 0 is unused.
// Returns 0 when the count would exceed 2^32.
inline uint64_t ep_count(int32_t depth, int32_t fanout) {
  uint64_t c = 1, level = 1;
  for (int32_t t = 0; t < depth; t++) {
    c += level;
    if (c > (1ull << 32)) return 0;
    level *= (uint64_t)fanout;
    if (level > (1ull << 32)) level = (1ull << 33);
  }
  return c;
}
inline uint64_t bytes_ep(int32_t depth, int32_t fanout) { return ep_count(depth, fanout) * 4; }

// Chain layout (the half-bounded index): the recorded prefix sizes that own
// a graph, s_0 = n, s_{i+1} = ceil(s_i / base), while s_i - 1 >= leaf.
// Depth i < K holds prefix [0, s_i - 1]; depth K + i the suffix
// [n - s_i, n - 1].  Rows are stored depth after depth, each depth's rows
// for its own positions only.
inline std::vector<int64_t> chain_sizes(int64_t n, int32_t leaf, int32_t base) {
  std::vector<int64_t> out;
  for (int64_t s = n; s - 1 >= leaf; s = (s + base - 1) / base) {
    out.push_back(s);
    if (s == 1) break;
  }
  return out;
}
// Row offset of position p at depth t is row_base[t] + p.
inline std::vector<int64_t> chain_row_base(int64_t n, const std::vector<int64_t>& sizes) {
  const size_t k = sizes.size();
  std::vector<int64_t> base(2 * k);
  int64_t off = 0;
  for (size_t t = 0; t < 2 * k; t++) {
    const int64_t sz = sizes[t % k];
    const int64_t start = t < k ? 0 : n - sz;
    base[t] = off - start;
    off += sz;
  }
  return base;
}
inline int64_t chain_rows(const std::vector<int64_t>& sizes) {
  int64_t r = 0;
  for (int64_t s : sizes) r += 2 * s;
  return r;
}

// Software CRC-32C (Castagnoli, reflected polynomial 0x82F63B78), eight
// bytes per step with slicing tables.
class Crc32c {
 public:
  Crc32c() {
    for (uint32_t i = 0; i < 256; i++) {
      uint32_t c = i;
      for (int k = 0; k < 8; k++) c = (c >> 1) ^ ((c & 1) ? 0x82F63B78u : 0u);
      t_[0][i] = c;
    }
    for (uint32_t i = 0; i < 256; i++)
      for (int s = 1; s < 8; s++) t_[s][i] = (t_[s - 1][i] >> 8) ^ t_[0][t_[s - 1][i] & 0xFF];
  }
  uint32_t update(uint32_t crc, const void* data, size_t len) const {
    const uint8_t* p = static_cast<const uint8_t*>(data);
    crc = ~crc;
    while (len >= 8) {
      uint64_t w;
      std::memcpy(&w, p, 8);
      w ^= crc;
      crc = t_[7][w & 0xFF] ^ t_[6][(w >> 8) & 0xFF] ^ t_[5][(w >> 16) & 0xFF] ^
            t_[4][(w >> 24) & 0xFF] ^ t_[3][(w >> 32) & 0xFF] ^ t_[2][(w >> 40) & 0xFF] ^
            t_[1][(w >> 48) & 0xFF] ^ t_[0][(w >> 56) & 0xFF];
      p += 8;
      len -= 8;
    }
    while (len--) crc = (crc >> 8) ^ t_[0][(crc ^ *p++) & 0xFF];
    return ~crc;
  }

 private:
  uint32_t t_[8][256];
};

inline const Crc32c& crc32c() {
  static const Crc32c c;
  return c;
}

}  // namespace esg
