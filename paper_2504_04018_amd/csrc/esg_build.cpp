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
#include "esg_gpu_build.h"

namespace {

using Cand = std::pair<float, uint32_t>;  // (squared distance, position)

// Squared Euclidean distance in float32 with the search kernels' fixed
// summation order, so that the host and the device builders compute the
// same values: the row is cut into chunks of 4 values, chunk c goes to lane
// c mod G (G = the chunk count rounded up to a power of two, at most 64),
// each lane accumulates fma(x - q, x - q, acc) over its chunks in order,
// and the lanes are added pairwise (lane t + lane t + s for s = 1, 2, 4, ...).
inline float l2sq(const float* x, const float* q, int d) {
  const int C = (d + 3) / 4;
  int G = 1;
  while (G < C) G <<= 1;
  if (G > 64) G = 64;
  float acc[64];
  for (int t = 0; t < G; t++) acc[t] = 0.0f;
  for (int c = 0; c < C; c++) {
    float a = acc[c & (G - 1)];
    const int j0 = 4 * c, j1 = std::min(d, j0 + 4);
    for (int j = j0; j < j1; j++) {
      const float t = x[j] - q[j];
      a = std::fma(t, t, a);
    }
    acc[c & (G - 1)] = a;
  }
  for (int s = 1; s < G; s <<= 1)
    for (int t = 0; t < G; t += 2 * s) acc[t] = acc[t] + acc[t + s];
  return acc[0];
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

// One insertion sequence: the graph on positions [a, cur-1] receives
// positions cur..end, then next_cur..next_end (a node whose first child is
// built from scratch inserts that child's points first).
struct Job {
  int64_t a = 0, cur = 0, end = -1, next_cur = 0, next_end = -1;
  uint32_t ep = 0;
  int64_t ep_size = 0;
};

struct Builder {
  int64_t n;
  int d, R, leaf, efc, batch_max, n_depth, verbose, fanout;
  const float* X;          // [n][d], position order
  uint32_t* adj;           // [n_depth][n][R]
  esgb::GpuState* gpu = nullptr;   // insertion rounds on a HIP device (null: host threads)
  bool gpu_ok = true;

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

  // Every sum runs in point order (per dimension) or dimension order (per
  // point), whatever the thread count, so the result does not depend on it.
  uint32_t medoid(int64_t a, int64_t b) const {
    const int64_t L = b - a + 1;
    const bool par = L * d >= (1 << 20);
    std::vector<double> mean((size_t)d, 0.0);
    constexpr int kCols = 16;
#pragma omp parallel for schedule(static) if (par)
    for (int j0 = 0; j0 < d; j0 += kCols) {
      const int j1 = std::min(d, j0 + kCols);
      double acc[kCols] = {};
      for (int64_t p = a; p <= b; p++)
        for (int j = j0; j < j1; j++) acc[j - j0] += (double)X[(size_t)p * d + j];
      for (int j = j0; j < j1; j++) mean[(size_t)j] = acc[j - j0] / (double)L;
    }
    double best = INFINITY;
    uint32_t arg = (uint32_t)a;
#pragma omp parallel if (par)
    {
      double tb = INFINITY;
      uint32_t ta = (uint32_t)a;
#pragma omp for schedule(static) nowait
      for (int64_t p = a; p <= b; p++) {
        double s = 0.0;
        for (int j = 0; j < d; j++) {
          const double t = (double)X[(size_t)p * d + j] - mean[(size_t)j];
          s += t * t;
        }
        if (s < tb) {   // static chunks in order: the first minimum of the chunk
          tb = s;
          ta = (uint32_t)p;
        }
      }
#pragma omp critical
      if (tb < best || (tb == best && ta < arg)) {
        best = tb;
        arg = ta;
      }
    }
    return arg;
  }

  // One insertion round against the frozen graph: every point pts[i] is
  // searched from eps[i] and pruned to at most R neighbours (all in
  // parallel), then the forward rows are written and the reverse edges
  // applied, one target at a time in (target, source) order.
  void round_cpu(uint32_t* rw, const std::vector<uint32_t>& pts, const std::vector<uint32_t>& eps) {
    const int64_t nb = (int64_t)pts.size();
    std::vector<uint32_t> sel((size_t)nb * R, ESG_NO_NODE);
#pragma omp parallel for schedule(dynamic, 1) if (nb > 1)
    for (int64_t i = 0; i < nb; i++) {
      // One visit-tag array per OS thread (nested regions run serialized).
      static thread_local VisitTags vt;
      static thread_local std::vector<Cand> cands;
      if ((int64_t)vt.tag.size() != n) vt.reset(n);
      search(rw, eps[(size_t)i], vec(pts[(size_t)i]), efc, vt, cands);
      occlude(cands, pts[(size_t)i], &sel[(size_t)i * R]);
    }
    std::vector<uint64_t> prop;   // (target << 32) | source
    for (int64_t i = 0; i < nb; i++) {
      const uint32_t p = pts[(size_t)i];
      std::memcpy(rw + (size_t)p * R, &sel[(size_t)i * R], sizeof(uint32_t) * R);
      for (int j = 0; j < R; j++) {
        const uint32_t c = sel[(size_t)i * R + j];
        if (c == ESG_NO_NODE) break;
        prop.push_back(((uint64_t)c << 32) | p);
      }
    }
    std::sort(prop.begin(), prop.end());
    std::vector<size_t> starts;
    for (size_t i = 0; i < prop.size(); i++)
      if (i == 0 || (prop[i] >> 32) != (prop[i - 1] >> 32)) starts.push_back(i);
    starts.push_back(prop.size());
    const int64_t n_groups = (int64_t)starts.size() - 1;
#pragma omp parallel for schedule(dynamic, 16) if (n_groups > 64)
    for (int64_t g = 0; g < n_groups; g++) {
      const size_t i0 = starts[(size_t)g], i1 = starts[(size_t)g + 1];
      const uint32_t c = (uint32_t)(prop[i0] >> 32);
      uint32_t* row = rw + (size_t)c * R;
      int len = row_len(row, R);
      if (len + (int)(i1 - i0) <= R) {
        for (size_t i = i0; i < i1; i++) row[len++] = (uint32_t)prop[i];
        continue;
      }
      std::vector<Cand> cands;
      cands.reserve((size_t)len + (i1 - i0));
      for (int j = 0; j < len; j++) cands.push_back({l2sq(vec(c), vec(row[j]), d), row[j]});
      for (size_t i = i0; i < i1; i++) {
        const uint32_t p = (uint32_t)prop[i];
        cands.push_back({l2sq(vec(c), vec(p), d), p});
      }
      std::sort(cands.begin(), cands.end());
      occlude(cands, c, row);
    }
  }

  // Runs insertion sequences in lockstep rounds: in each round every
  // unfinished job inserts its next batch, whose size depends only on the
  // job's current graph size.  Jobs write disjoint rows, so each one ends
  // as it would alone.  The entry point of a job's searches is the medoid
  // of its current graph, refreshed whenever the graph has doubled.
  void insert_jobs(int depth, uint32_t* rw, std::vector<Job>& jobs) {
    std::vector<uint32_t> pts, eps, lo, hi;
    for (;;) {
      std::vector<size_t> act;
      for (size_t j = 0; j < jobs.size(); j++) {
        Job& J = jobs[j];
        if (J.cur > J.end && J.next_cur <= J.next_end) {
          J.cur = J.next_cur;
          J.end = J.next_end;
          J.next_end = J.next_cur - 1;
          J.ep_size = 0;
        }
        if (J.cur <= J.end) act.push_back(j);
      }
      if (act.empty()) break;
#pragma omp parallel for schedule(dynamic, 1) if (act.size() > 1)
      for (size_t u = 0; u < act.size(); u++) {
        Job& J = jobs[act[u]];
        const int64_t size = J.cur - J.a;
        if (size >= 2 * J.ep_size + 1 || J.ep_size == 0) {
          J.ep = medoid(J.a, J.cur - 1);
          J.ep_size = size;
        }
      }
      pts.clear();
      eps.clear();
      lo.clear();
      hi.clear();
      for (size_t j : act) {
        Job& J = jobs[j];
        int64_t B = std::max<int64_t>(1, std::min<int64_t>((J.cur - J.a) / 16, batch_max));
        B = std::min<int64_t>(B, J.end - J.cur + 1);
        for (int64_t i = 0; i < B; i++) {
          pts.push_back((uint32_t)(J.cur + i));
          eps.push_back(J.ep);
          lo.push_back((uint32_t)J.a);
          hi.push_back((uint32_t)(J.cur - 1));
        }
        J.cur += B;
      }
      if (gpu) {
        if (!gpu_ok) continue;
        if (esgb::gpu_round(gpu, depth, (int64_t)pts.size(), pts.data(), eps.data(), lo.data(),
                            hi.data()) != ESG_OK)
          gpu_ok = false;
      } else {
        round_cpu(rw, pts, eps);
      }
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

  // The insertion job of node [a,b] at depth t (Alg. 3): its first child's
  // graph is copied from depth t+1 when that child owns one; otherwise the
  // first child is built from scratch from its first point.  Then the
  // remaining points are inserted.
  Job node_job(int t, int64_t a, int64_t b) {
    const int64_t mid = child_start(a, b - a + 1, fanout, 1) - 1;   // end of the first child
    Job J;
    J.a = a;
    if (mid - a >= leaf) {
      if (gpu) {
        if (gpu_ok && esgb::gpu_copy_rows(gpu, t, t + 1, a, mid - a + 1) != ESG_OK) gpu_ok = false;
      } else {
        std::memcpy(rows(t) + (size_t)a * R, rows(t + 1) + (size_t)a * R,
                    sizeof(uint32_t) * (size_t)R * (size_t)(mid - a + 1));
      }
      J.cur = mid + 1;
      J.end = b;
    } else {
      J.cur = a + 1;
      J.end = mid;
      J.next_cur = mid + 1;
      J.next_end = b;
    }
    return J;
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
  if (B.gpu && B.gpu_ok && esgb::gpu_reset(B.gpu, B.X) != ESG_OK) B.gpu_ok = false;
  int64_t done = 0;                     // positions [0, done) inserted
  for (size_t j = k; j-- > 0;) {
    const int64_t s = sizes[j];
    std::vector<Job> jobs(1);
    jobs[0].a = 0;
    jobs[0].cur = done == 0 ? 1 : done;
    jobs[0].end = s - 1;
    B.insert_jobs(0, W.data(), jobs);
    if (B.gpu && B.gpu_ok && esgb::gpu_get_rows(B.gpu, 0, W.data()) != ESG_OK) B.gpu_ok = false;
    done = s;
    const uint32_t e = B.medoid(0, s - 1);
    B.repair(0, 0, s - 1, e);
    if (B.gpu && B.gpu_ok && esgb::gpu_put_rows(B.gpu, 0, W.data()) != ESG_OK) B.gpu_ok = false;
    eps[j] = e;
    snapshot(j, s);                     // record the graph of [0, s - 1] now
    if (B.verbose)
      fprintf(stderr, "[esg_build] chain prefix of %lld points recorded\n", (long long)s);
    (void)R;
  }
}

// Owns the device state of a GPU build.
struct GpuHolder {
  esgb::GpuState* g = nullptr;
  ~GpuHolder() {
    if (g) esgb::gpu_close(g);
  }
};

// Points of one device insertion round at most, and the largest batch of
// one node on the device (its reverse-edge groups are sorted in LDS).
constexpr int64_t kGpuRound = 65536;
constexpr int32_t kGpuBatchMax = 8192;

int32_t build_chains(const float* X, const std::vector<int64_t>& order,
                     const std::vector<double>& sorted_attr, int64_t n, int32_t d,
                     const esg_build_params& P, int fanout, const MetricInfo& mi,
                     const char* out_path, int32_t device) {
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
  GpuHolder gh;
  if (device >= 0) {
    const int32_t st = esgb::gpu_open(device, X, n, d, R, 1, B.efc, kGpuRound, &gh.g);
    if (st != ESG_OK) return st;
    B.gpu = gh.g;
  }
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
  if (!B.gpu_ok) return ESG_EHIP;
  return write_index(out_path, n, d, P, fanout, (int)(2 * k), 1, mi, order.data(),
                     sorted_attr.data(), X, adj, ep);
}

}  // namespace

static int32_t build_impl(const float* vecs, const double* attr, int64_t n, int32_t d,
                   const esg_build_params* params, int32_t device, const char* out_path) {
  if (!vecs || !attr || !params || !out_path || n <= 0 || n >= (int64_t)ESG_NO_NODE || d <= 0)
    return ESG_EINVAL;
  const esg_build_params& P = *params;
  if (P.degree < 1 || P.degree > ESG_DEGREE_MAX || P.leaf < 1 || P.ef_construction < 1 ||
      P.fanout < 0 || P.fanout == 1 || P.layout < 0 || P.layout > 1 ||
      P.metric < ESG_METRIC_L2 || P.metric > ESG_METRIC_IP || d >= 65536)
    return ESG_EINVAL;
  const int fanout = P.fanout == 0 ? 2 : P.fanout;
  if (fanout > ESG_FANOUT_MAX) return ESG_EUNSUPPORTED;
  if (device >= 0 && P.batch_max > kGpuBatchMax) return ESG_EINVAL;
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
      return build_chains(X.data(), order, sorted_attr, n, ds, P, fanout, mi, out_path, device);
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
    GpuHolder gh;
    if (device >= 0 && n_depth > 0) {
      const int32_t st =
          esgb::gpu_open(device, X.data(), n, ds, B.R, n_depth, B.efc, kGpuRound, &gh.g);
      if (st != ESG_OK) return st;
      B.gpu = gh.g;
    }

    std::vector<uint32_t> ep((size_t)esg::ep_count(n_depth, fanout), ESG_NO_NODE);
    for (int t = n_depth - 1; t >= 0; t--) {
      std::vector<NodeRef> level;
      for (const NodeRef& nd : nodes)
        if (nd.depth == t) level.push_back(nd);
      std::vector<Job> jobs;
      for (const NodeRef& nd : level) jobs.push_back(B.node_job(t, nd.a, nd.b));
      B.insert_jobs(t, B.rows(t), jobs);
      if (B.gpu && B.gpu_ok && esgb::gpu_get_rows(B.gpu, t, B.rows(t)) != ESG_OK) B.gpu_ok = false;
      if (!B.gpu_ok) return ESG_EHIP;
      int64_t repaired = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : repaired)
      for (int64_t i = 0; i < (int64_t)level.size(); i++) {
        const NodeRef& nd = level[(size_t)i];
        const uint32_t e = B.medoid(nd.a, nd.b);
        ep[(size_t)nd.heap] = e;
        repaired += B.repair(t, nd.a, nd.b, e);
      }
      if (B.gpu && esgb::gpu_put_rows(B.gpu, t, B.rows(t)) != ESG_OK) return ESG_EHIP;
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

extern "C" int32_t esg_build_index(const float* vecs, const double* attr, int64_t n, int32_t d,
                                   const esg_build_params* params, const char* out_path) {
  return build_impl(vecs, attr, n, d, params, -1, out_path);
}

extern "C" int32_t esg_build_index_gpu(const float* vecs, const double* attr, int64_t n, int32_t d,
                                       const esg_build_params* params, int32_t hip_device,
                                       const char* out_path) {
  if (hip_device < 0) return ESG_EINVAL;
  return build_impl(vecs, attr, n, d, params, hip_device, out_path);
}
