// Host builder of the HBI-2D elastic-graph index (Section 4.2, Alg. 3).
//
// The segment tree over positions [0, n-1] splits node [a,b] of L points
// into `fanout` children, child j = [a + ceil(jL/f), a + ceil((j+1)L/f) - 1]
// (at fanout 2: [a, floor((a+b)/2)] and the rest, as in Alg. 3; larger
// fanouts are the extension of Section 4.2).  A node with b - a >= leaf owns
// a proximity graph; its graph is a copy of its first child's graph plus
// the insertion of the remaining points (Alg. 3); when the first child is a
// leaf its graph is first built from scratch.  Every graph of one tree
// depth covers disjoint positions, so the graphs of depth t share one
// adjacency array adj[t][n][R].
//
// Insertion follows the graph-index construction recalled in Section 2.1:
// a beam search of width ef_construction finds candidates, edge occlusion
// keeps at most R of them (a candidate c is dropped when an already kept
// neighbour s is closer to c than the new point is), and reverse edges are
// added, re-pruning a full list with the same rule.  Points are inserted in
// batches whose size depends only on the current graph size: the searches
// of one batch run in parallel against the graph as it was before the
// batch, then all edge updates are applied in a fixed order.  The output is
// therefore independent of the thread count.
//
// The entry point of each node graph is its medoid: the point nearest (in
// float64) to the mean of the node's points, ties to the smaller position.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <queue>
#include <utility>
#include <vector>

#include "../../include/esg.h"
#include "esg_format.h"

namespace {

using Cand = std::pair<float, uint32_t>;  // (squared distance, position)

inline float l2sq(const float* a, const float* b, int d) {
  float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int j = 0;
  for (; j + 8 <= d; j += 8) {
    for (int e = 0; e < 8; e++) {
      float t = a[j + e] - b[j + e];
      acc[e] += t * t;
    }
  }
  float s = 0.f;
  for (; j < d; j++) {
    float t = a[j] - b[j];
    s += t * t;
  }
  return s + ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

struct VisitTags {
  std::vector<uint32_t> tag;
  uint32_t cur = 0;
  void reset(int64_t n) {
    tag.assign((size_t)n, 0);
    cur = 0;
  }
  void next() {
    if (++cur == 0) {
      std::fill(tag.begin(), tag.end(), 0);
      cur = 1;
    }
  }
};

// First position of child j of the node starting at a with L points.
inline int64_t child_start(int64_t a, int64_t L, int f, int64_t j) { return a + (j * L + f - 1) / f; }

struct Builder {
  int64_t n;
  int d, R, leaf, efc, batch_max, n_depth, verbose, fanout;
  const float* X;          // [n][d], position order
  uint32_t* adj;           // [n_depth][n][R]

  uint32_t* rows(int t) { return adj + (size_t)t * (size_t)n * (size_t)R; }
  const float* vec(uint32_t p) const { return X + (size_t)p * (size_t)d; }

  static int row_len(const uint32_t* row, int R) {
    int c = 0;
    while (c < R && row[c] != ESG_NO_NODE) c++;
    return c;
  }

  // Beam search over the graph `rw` (rows hold global positions) from ep.
  void search(const uint32_t* rw, uint32_t ep, const float* q, int ef, VisitTags& vt,
              std::vector<Cand>& out) const {
    vt.next();
    std::priority_queue<Cand, std::vector<Cand>, std::greater<Cand>> cand;  // min
    std::priority_queue<Cand> res;                                          // max
    Cand e{l2sq(vec(ep), q, d), ep};
    vt.tag[ep] = vt.cur;
    cand.push(e);
    res.push(e);
    while (!cand.empty()) {
      Cand c = cand.top();
      if ((int)res.size() >= ef && res.top() < c) break;
      cand.pop();
      const uint32_t* row = rw + (size_t)c.second * R;
      for (int s = 0; s < R; s++) {
        uint32_t v = row[s];
        if (v == ESG_NO_NODE) break;
        if (vt.tag[v] == vt.cur) continue;
        vt.tag[v] = vt.cur;
        Cand nv{l2sq(vec(v), q, d), v};
        if ((int)res.size() < ef || nv < res.top()) {
          cand.push(nv);
          res.push(nv);
          if ((int)res.size() > ef) res.pop();
        }
      }
    }
    out.resize(res.size());
    for (size_t i = res.size(); i-- > 0;) {
      out[i] = res.top();
      res.pop();
    }
  }

  // Edge occlusion over candidates sorted ascending by distance to the base point.
  int occlude(const std::vector<Cand>& cands, uint32_t self, uint32_t* out) const {
    int m = 0;
    for (const Cand& c : cands) {
      if (m >= R) break;
      if (c.second == self) continue;
      bool keep = true;
      for (int s = 0; s < m; s++) {
        if (l2sq(vec(c.second), vec(out[s]), d) < c.first) {
          keep = false;
          break;
        }
      }
      if (keep) out[m++] = c.second;
    }
    for (int s = m; s < R; s++) out[s] = ESG_NO_NODE;
    return m;
  }

  uint32_t medoid(int64_t a, int64_t b) const {
    std::vector<double> mean((size_t)d, 0.0);
    for (int64_t p = a; p <= b; p++)
      for (int j = 0; j < d; j++) mean[j] += (double)X[(size_t)p * d + j];
    for (int j = 0; j < d; j++) mean[j] /= (double)(b - a + 1);
    double best = INFINITY;
    uint32_t arg = (uint32_t)a;
    for (int64_t p = a; p <= b; p++) {
      double s = 0.0;
      for (int j = 0; j < d; j++) {
        double t = (double)X[(size_t)p * d + j] - mean[j];
        s += t * t;
      }
      if (s < best) {
        best = s;
        arg = (uint32_t)p;
      }
    }
    return arg;
  }

  // Graph on [a, s-1] (rows of `rw`) receives positions s..e.
  void insert_range(uint32_t* rw, int64_t a, int64_t s, int64_t e, bool par) {
    int64_t cur = s;
    int64_t ep_size = 0;
    uint32_t ep = (uint32_t)a;
    std::vector<std::vector<uint32_t>> sel;
    std::vector<std::pair<uint64_t, float>> prop;  // ((target<<32)|source, dist)
    while (cur <= e) {
      int64_t size = cur - a;
      if (size >= 2 * ep_size + 1 || ep_size == 0) {
        ep = medoid(a, cur - 1);
        ep_size = size;
      }
      int64_t B = std::max<int64_t>(1, std::min<int64_t>(size / 16, batch_max));
      B = std::min<int64_t>(B, e - cur + 1);
      sel.assign((size_t)B, std::vector<uint32_t>((size_t)R, ESG_NO_NODE));
      // 1) searches against the frozen graph
#pragma omp parallel for schedule(dynamic, 1) if (par && B > 1)
      for (int64_t i = 0; i < B; i++) {
        std::vector<Cand> cands;
        uint32_t p = (uint32_t)(cur + i);
        // One visit-tag array per OS thread: omp_get_thread_num() is 0 inside
        // the serialized inner region of every outer thread, so it cannot
        // index per-thread state here.
        static thread_local VisitTags vt;
        if ((int64_t)vt.tag.size() != n) vt.reset(n);
        search(rw, ep, vec(p), efc, vt, cands);
        occlude(cands, p, sel[(size_t)i].data());
      }
      // 2) forward edges and reverse-edge proposals, in position order
      prop.clear();
      for (int64_t i = 0; i < B; i++) {
        uint32_t p = (uint32_t)(cur + i);
        std::memcpy(rw + (size_t)p * R, sel[(size_t)i].data(), sizeof(uint32_t) * R);
        for (int j = 0; j < R; j++) {
          uint32_t c = sel[(size_t)i][(size_t)j];
          if (c == ESG_NO_NODE) break;
          prop.push_back({((uint64_t)c << 32) | p, 0.f});
        }
      }
      std::sort(prop.begin(), prop.end());
      // group boundaries per target
      std::vector<size_t> starts;
      for (size_t i = 0; i < prop.size(); i++)
        if (i == 0 || (prop[i].first >> 32) != (prop[i - 1].first >> 32)) starts.push_back(i);
      starts.push_back(prop.size());
      // 3) reverse edges, one target per iteration (targets are distinct)
      const int64_t n_groups = (int64_t)starts.size() - 1;
#pragma omp parallel for schedule(dynamic, 16) if (par && n_groups > 64)
      for (int64_t g = 0; g < n_groups; g++) {
        size_t i0 = starts[(size_t)g], i1 = starts[(size_t)g + 1];
        uint32_t c = (uint32_t)(prop[i0].first >> 32);
        uint32_t* row = rw + (size_t)c * R;
        int len = row_len(row, R);
        if (len + (int)(i1 - i0) <= R) {
          for (size_t i = i0; i < i1; i++) row[len++] = (uint32_t)(prop[i].first & 0xFFFFFFFFu);
          continue;
        }
        std::vector<Cand> cands;
        cands.reserve((size_t)len + (i1 - i0));
        for (int j = 0; j < len; j++) cands.push_back({l2sq(vec(c), vec(row[j]), d), row[j]});
        for (size_t i = i0; i < i1; i++) {
          uint32_t p = (uint32_t)(prop[i].first & 0xFFFFFFFFu);
          cands.push_back({l2sq(vec(c), vec(p), d), p});
        }
        std::sort(cands.begin(), cands.end());
        occlude(cands, c, row);
      }
      cur += B;
    }
  }

  // Connectivity repair of the graph of node [a,b] at depth t: every point
  // must be reachable from the entry e, so that a search with a beam as large
  // as the node visits all of it (Finding 1: the superset graph then answers
  // the sub-range exactly).  Occlusion pruning of reverse edges can leave a
  // point without in-edges.  Each round walks the graph from e and gives
  // every unreachable point u (in position order) an in-edge from a
  // reachable point v: the nearest reachable point with a free row slot
  // among u's neighbours and their neighbours, else u's nearest reachable
  // neighbour (its last slot is overwritten; a later round repairs whatever
  // that cuts off), else the nearest reachable point of the node with a free
  // slot.  Sequential and in a fixed order, so the result is deterministic.
  // Returns the number of edges added.
  int64_t repair(int t, int64_t a, int64_t b, uint32_t e) {
    uint32_t* rw = rows(t);
    const int64_t L = b - a + 1;
    std::vector<uint8_t> reach((size_t)L);
    std::vector<uint32_t> queue;
    int64_t added = 0;
    for (int round = 0; round < 64; round++) {
      std::fill(reach.begin(), reach.end(), 0);
      queue.clear();
      queue.push_back(e);
      reach[(size_t)(e - a)] = 1;
      for (size_t i = 0; i < queue.size(); i++) {
        const uint32_t* row = rw + (size_t)queue[i] * R;
        for (int s = 0; s < R && row[s] != ESG_NO_NODE; s++)
          if (!reach[(size_t)(row[s] - a)]) {
            reach[(size_t)(row[s] - a)] = 1;
            queue.push_back(row[s]);
          }
      }
      if ((int64_t)queue.size() == L) break;
      const bool last_resort = round >= 48;
      for (int64_t u = a; u <= b; u++) {
        if (reach[(size_t)(u - a)]) continue;
        const float* xu = vec((uint32_t)u);
        uint32_t best = ESG_NO_NODE, near = ESG_NO_NODE;
        float bd = INFINITY, nd = INFINITY;
        auto consider = [&](uint32_t v) {
          if (v == ESG_NO_NODE || !reach[(size_t)(v - a)]) return;
          const float dv = l2sq(xu, vec(v), d);
          if (dv < nd || (dv == nd && v < near)) { nd = dv; near = v; }
          if (row_len(rw + (size_t)v * R, R) < R && (dv < bd || (dv == bd && v < best))) {
            bd = dv;
            best = v;
          }
        };
        const uint32_t* ru = rw + (size_t)u * R;
        for (int s = 0; s < R && ru[s] != ESG_NO_NODE; s++) {
          consider(ru[s]);
          const uint32_t* r2 = rw + (size_t)ru[s] * R;
          for (int s2 = 0; s2 < R && r2[s2] != ESG_NO_NODE; s2++) consider(r2[s2]);
        }
        if (best == ESG_NO_NODE && (near == ESG_NO_NODE || last_resort)) {
          for (int64_t v = a; v <= b; v++) consider((uint32_t)v);
        }
        uint32_t v = best != ESG_NO_NODE ? best : near;
        if (v == ESG_NO_NODE) continue;
        uint32_t* rv = rw + (size_t)v * R;
        const int len = row_len(rv, R);
        rv[len < R ? len : R - 1] = (uint32_t)u;
        added++;
      }
    }
    return added;
  }

  void build_node(int t, int64_t a, int64_t b, bool par) {
    const int64_t mid = child_start(a, b - a + 1, fanout, 1) - 1;   // end of the first child
    uint32_t* rw = rows(t);
    if (mid - a >= leaf) {
      // first child owns a graph at depth t+1: copy it
      std::memcpy(rw + (size_t)a * R, rows(t + 1) + (size_t)a * R,
                  sizeof(uint32_t) * (size_t)R * (size_t)(mid - a + 1));
    } else {
      // build the left half from scratch, starting from its first point
      for (int j = 0; j < R; j++) rw[(size_t)a * R + j] = ESG_NO_NODE;
      if (mid > a) insert_range(rw, a, a + 1, mid, par);
    }
    insert_range(rw, a, mid + 1, b, par);
  }
};

struct NodeRef {
  int depth;
  int64_t heap, a, b;
};

void collect(int64_t a, int64_t b, int depth, int64_t heap, int leaf, int f,
             std::vector<NodeRef>& out) {
  if (b - a < leaf) return;
  out.push_back({depth, heap, a, b});
  for (int64_t j = 0; j < f; j++) {
    const int64_t ca = child_start(a, b - a + 1, f, j), cb = child_start(a, b - a + 1, f, j + 1) - 1;
    if (ca <= cb) collect(ca, cb, depth + 1, (int64_t)f * (heap - 1) + 2 + j, leaf, f, out);
  }
}

bool write_all(FILE* f, const void* p, uint64_t bytes) {
  const char* c = static_cast<const char*>(p);
  while (bytes > 0) {
    size_t chunk = (size_t)std::min<uint64_t>(bytes, 1ull << 30);
    if (fwrite(c, 1, chunk, f) != chunk) return false;
    c += chunk;
    bytes -= chunk;
  }
  return true;
}

bool pad_to(FILE* f, uint64_t off) {
  long pos = ftell(f);
  if (pos < 0) return false;
  static const char zeros[4096] = {0};
  uint64_t cur = (uint64_t)pos;
  while (cur < off) {
    size_t chunk = (size_t)std::min<uint64_t>(off - cur, sizeof(zeros));
    if (fwrite(zeros, 1, chunk, f) != chunk) return false;
    cur += chunk;
  }
  return true;
}

// What the stored vectors were made from (esg.h, ESG_METRIC_*).
struct MetricInfo {
  int32_t metric = ESG_METRIC_L2, dq = 0;
  double max_norm2 = 0.0;
};

// Writes the index file (layout documented in esg.h).
int32_t write_index(const char* out_path, int64_t n, int32_t d, const esg_build_params& P,
                    int fanout, int n_depth, int layout, const MetricInfo& mi, const int64_t* ids,
                    const double* attr, const float* X, const std::vector<uint32_t>& adj,
                    const std::vector<uint32_t>& ep) {
  const uint64_t adj_bytes = (uint64_t)adj.size() * 4, ep_bytes = (uint64_t)ep.size() * 4;
  esg::FileHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, esg::kMagic, 8);
  h.version = esg::kVersion;
  h.header_bytes = esg::kHeaderBytes;
  h.n = n;
  h.d = d;
  h.degree = P.degree;
  h.leaf = P.leaf;
  h.fanout = fanout;
  h.n_depth = n_depth;
  h.c_den = fanout;   // elastic constant c = 1/fanout (Lemma 4.3; Lemma 4.1 with base B)
  h.layout = layout;
  h.ef_construction = P.ef_construction;
  h.metric = mi.metric;
  h.dq = mi.dq;
  h.max_norm2 = mi.max_norm2;
  h.off_ids = esg::align_up(esg::kHeaderBytes);
  h.off_attr = esg::align_up(h.off_ids + esg::bytes_ids(n));
  h.off_vec = esg::align_up(h.off_attr + esg::bytes_attr(n));
  h.off_adj = esg::align_up(h.off_vec + esg::bytes_vec(n, d));
  h.off_ep = esg::align_up(h.off_adj + adj_bytes);
  h.file_bytes = h.off_ep + ep_bytes;
  const esg::Crc32c& crc = esg::crc32c();
  h.crc_sections[0] = crc.update(0, ids, esg::bytes_ids(n));
  h.crc_sections[1] = crc.update(0, attr, esg::bytes_attr(n));
  h.crc_sections[2] = crc.update(0, X, esg::bytes_vec(n, d));
  h.crc_sections[3] = crc.update(0, adj.data(), adj_bytes);
  h.crc_sections[4] = crc.update(0, ep.data(), ep_bytes);
  h.crc_header = crc.update(0, &h, offsetof(esg::FileHeader, crc_header));

  FILE* f = fopen(out_path, "wb");
  if (!f) return ESG_EIO;
  bool ok = write_all(f, &h, sizeof(h)) && pad_to(f, h.off_ids) &&
            write_all(f, ids, esg::bytes_ids(n)) && pad_to(f, h.off_attr) &&
            write_all(f, attr, esg::bytes_attr(n)) && pad_to(f, h.off_vec) &&
            write_all(f, X, esg::bytes_vec(n, d)) && pad_to(f, h.off_adj) &&
            write_all(f, adj.data(), adj_bytes) &&
            pad_to(f, h.off_ep) && write_all(f, ep.data(), ep_bytes);
  ok = (fclose(f) == 0) && ok;
  return ok ? ESG_OK : ESG_EIO;
}

// Half-bounded index (Section 4.1, Alg. 2): the points are inserted in
// position order into one graph, and the graph is recorded each time the
// inserted prefix reaches a recorded size s_i (smallest first); the suffix
// chain does the same in decreasing position order (built on the mirrored
// positions p -> n-1-p and mapped back).  Each recorded graph gets its
// medoid entry and the reachability repair before the insertion goes on.
template <typename Snapshot>
void build_chain(Builder& B, const std::vector<int64_t>& sizes, std::vector<uint32_t>& W,
                 std::vector<uint32_t>& eps, Snapshot snapshot) {
  const int R = B.R;
  const size_t k = sizes.size();
  eps.assign(k, ESG_NO_NODE);
  std::fill(W.begin(), W.end(), ESG_NO_NODE);
  B.adj = W.data();
  int64_t done = 0;                     // positions [0, done) inserted
  for (size_t j = k; j-- > 0;) {
    const int64_t s = sizes[j];
    if (done == 0) {
      if (s > 1) B.insert_range(W.data(), 0, 1, s - 1, true);
    } else if (s > done) {
      B.insert_range(W.data(), 0, done, s - 1, true);
    }
    done = s;
    const uint32_t e = B.medoid(0, s - 1);
    B.repair(0, 0, s - 1, e);
    eps[j] = e;
    snapshot(j, s);                     // record the graph of [0, s - 1] now
    if (B.verbose)
      fprintf(stderr, "[esg_build] chain prefix of %lld points recorded\n", (long long)s);
    (void)R;
  }
}

int32_t build_chains(const float* X, const std::vector<int64_t>& order,
                     const std::vector<double>& sorted_attr, int64_t n, int32_t d,
                     const esg_build_params& P, int fanout, const MetricInfo& mi,
                     const char* out_path) {
  const std::vector<int64_t> sizes = esg::chain_sizes(n, P.leaf, fanout);
  const size_t k = sizes.size();
  if (k == 0 || 2 * k > 40) return ESG_ERANGE;
  const int R = P.degree;
  Builder B;
  B.n = n;
  B.d = d;
  B.R = R;
  B.leaf = P.leaf;
  B.efc = P.ef_construction;
  B.batch_max = P.batch_max > 0 ? P.batch_max : 1024;
  B.n_depth = 1;
  B.verbose = P.verbose;
  B.fanout = fanout;
  std::vector<uint32_t> W((size_t)n * R), eps_p, eps_s;
  const std::vector<int64_t> row_base = esg::chain_row_base(n, sizes);
  std::vector<uint32_t> adj((size_t)esg::chain_rows(sizes) * R, ESG_NO_NODE);
  // prefixes
  B.X = X;
  build_chain(B, sizes, W, eps_p, [&](size_t i, int64_t s) {
    std::memcpy(&adj[(size_t)row_base[i] * R], W.data(), sizeof(uint32_t) * R * (size_t)s);
  });
  // suffixes on the mirrored positions p -> n-1-p
  std::vector<float> Xr((size_t)n * d);
  for (int64_t p = 0; p < n; p++)
    std::memcpy(&Xr[(size_t)p * d], X + (size_t)(n - 1 - p) * d, sizeof(float) * d);
  B.X = Xr.data();
  build_chain(B, sizes, W, eps_s, [&](size_t i, int64_t s) {
    const size_t t = k + i;
    for (int64_t p = n - s; p < n; p++) {
      const uint32_t* src = &W[(size_t)(n - 1 - p) * R];
      uint32_t* dst = &adj[(size_t)(row_base[t] + p) * R];
      for (int j = 0; j < R; j++)
        dst[j] = src[j] == ESG_NO_NODE ? ESG_NO_NODE : (uint32_t)(n - 1 - (int64_t)src[j]);
    }
  });
  std::vector<uint32_t> ep(2 * k + 1, ESG_NO_NODE);   // node number = depth + 1
  for (size_t i = 0; i < k; i++) {
    ep[1 + i] = eps_p[i];
    ep[1 + k + i] = (uint32_t)(n - 1 - (int64_t)eps_s[i]);
  }
  return write_index(out_path, n, d, P, fanout, (int)(2 * k), 1, mi, order.data(),
                     sorted_attr.data(), X, adj, ep);
}

}  // namespace

extern "C" int32_t esg_build_index(const float* vecs, const double* attr, int64_t n, int32_t d,
                                   const esg_build_params* params, const char* out_path) {
  if (!vecs || !attr || !params || !out_path || n <= 0 || n >= (int64_t)ESG_NO_NODE || d <= 0)
    return ESG_EINVAL;
  const esg_build_params& P = *params;
  if (P.degree < 1 || P.degree > ESG_DEGREE_MAX || P.leaf < 1 || P.ef_construction < 1 ||
      P.fanout < 0 || P.fanout == 1 || P.layout < 0 || P.layout > 1 ||
      P.metric < ESG_METRIC_L2 || P.metric > ESG_METRIC_IP || d >= 65536)
    return ESG_EINVAL;
  const int fanout = P.fanout == 0 ? 2 : P.fanout;
  if (fanout > ESG_FANOUT_MAX) return ESG_EUNSUPPORTED;
  for (int64_t i = 0; i < n; i++)
    if (std::isnan(attr[i])) return ESG_EINVAL;
  try {
    int nthreads = P.threads > 0 ? P.threads : omp_get_max_threads();
    omp_set_num_threads(nthreads);

    // Re-rank by attribute: position p holds the p-th smallest value.
    std::vector<int64_t> order((size_t)n);
    for (int64_t i = 0; i < n; i++) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t u, int64_t v) { return attr[u] < attr[v]; });
    std::vector<double> sorted_attr((size_t)n);
    MetricInfo mi;
    mi.metric = P.metric;
    mi.dq = d;
    // Other metrics become squared Euclidean distance over transformed
    // vectors: unit rows (angular), or one extra coordinate that brings
    // every row to norm M (inner product, the Euclidean transform of
    // Bachrach et al. 2014).  Norms are summed in float64.
    std::vector<double> norm2((size_t)n);
    bool bad = false;
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (int64_t i = 0; i < n; i++) {
      const float* v = vecs + (size_t)i * d;
      double s2 = 0.0;
      for (int32_t j = 0; j < d; j++) s2 += (double)v[j] * (double)v[j];
      norm2[(size_t)i] = s2;
      bad = bad || !std::isfinite(s2) || (P.metric == ESG_METRIC_ANGULAR && s2 == 0.0);
    }
    if (bad && P.metric != ESG_METRIC_L2) return ESG_EINVAL;
    if (P.metric == ESG_METRIC_IP)
      for (int64_t i = 0; i < n; i++) mi.max_norm2 = std::max(mi.max_norm2, norm2[(size_t)i]);
    const int32_t ds = P.metric == ESG_METRIC_IP ? d + 1 : d;   // stored length
    std::vector<float> X((size_t)n * (size_t)ds);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; p++) {
      const int64_t i = order[(size_t)p];
      sorted_attr[(size_t)p] = attr[i];
      const float* src = vecs + (size_t)i * d;
      float* dst = &X[(size_t)p * ds];
      if (P.metric == ESG_METRIC_ANGULAR) {
        const double inv = 1.0 / std::sqrt(norm2[(size_t)i]);
        for (int32_t j = 0; j < d; j++) dst[j] = (float)((double)src[j] * inv);
      } else {
        std::memcpy(dst, src, sizeof(float) * d);
      }
      if (P.metric == ESG_METRIC_IP)
        dst[d] = (float)std::sqrt(std::max(mi.max_norm2 - norm2[(size_t)i], 0.0));
    }

    if (P.layout == 1)
      return build_chains(X.data(), order, sorted_attr, n, ds, P, fanout, mi, out_path);
    std::vector<NodeRef> nodes;
    collect(0, n - 1, 0, 1, P.leaf, fanout, nodes);
    int n_depth = 0;
    for (const NodeRef& nd : nodes) n_depth = std::max(n_depth, nd.depth + 1);
    if (n_depth > 40 || esg::ep_count(n_depth, fanout) == 0) return ESG_ERANGE;

    Builder B;
    B.n = n;
    B.d = ds;
    B.R = P.degree;
    B.leaf = P.leaf;
    B.efc = P.ef_construction;
    B.batch_max = P.batch_max > 0 ? P.batch_max : 1024;
    B.n_depth = n_depth;
    B.verbose = P.verbose;
    B.fanout = fanout;
    B.X = X.data();
    std::vector<uint32_t> adj((size_t)n_depth * (size_t)n * (size_t)P.degree, ESG_NO_NODE);
    B.adj = adj.data();

    std::vector<uint32_t> ep((size_t)esg::ep_count(n_depth, fanout), ESG_NO_NODE);
    for (int t = n_depth - 1; t >= 0; t--) {
      std::vector<NodeRef> level;
      for (const NodeRef& nd : nodes)
        if (nd.depth == t) level.push_back(nd);
      bool outer = (int64_t)level.size() >= 2 * (int64_t)nthreads;
      if (outer) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t i = 0; i < (int64_t)level.size(); i++)
          B.build_node(t, level[(size_t)i].a, level[(size_t)i].b, false);
      } else {
        for (const NodeRef& nd : level) B.build_node(t, nd.a, nd.b, true);
      }
      int64_t repaired = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : repaired)
      for (int64_t i = 0; i < (int64_t)level.size(); i++) {
        const NodeRef& nd = level[(size_t)i];
        const uint32_t e = B.medoid(nd.a, nd.b);
        ep[(size_t)nd.heap] = e;
        repaired += B.repair(t, nd.a, nd.b, e);
      }
      if (P.verbose)
        fprintf(stderr, "[esg_build] depth %d: %zu graph nodes, %lld edges added for reachability\n",
                t, level.size(), (long long)repaired);
    }

    return write_index(out_path, n, ds, P, fanout, n_depth, 0, mi, order.data(), sorted_attr.data(),
                       X.data(), adj, ep);
  } catch (const std::bad_alloc&) {
    return ESG_ENOMEM;
  } catch (...) {
    return ESG_EINVAL;
  }
}
