/*
 * esg_oracle.c -- plain, slow, obviously-correct CPU oracle for ESG
 * range-filtered approximate k-NN search (Yang et al., "ESG: Elastic Graphs
 * for Range-Filtering Approximate k-Nearest Neighbor Search").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * timing do.  It shares no code, header, table or helper with the HIP path.
 *
 * What each function follows:
 *   oracle_select        Alg. 4 (Query-2D-Index) recursion, Section 4.2, with
 *                        the elastic test of Def. 3.1 at c = 1/c_den, for a
 *                        segment tree of fanout f (Section 4.2, Extensions).
 *   oracle_select_1d     the query rule of the half-bounded index (Section
 *                        4.1, Lemma 4.1): the tightest recorded prefix
 *                        [0, s-1] holding [0, r] (or suffix holding [l, N-1]),
 *                        recorded sizes s_0 = N, s_{i+1} = ceil(s_i / B).
 *   oracle_elastic_ok    Def. 3.1 test |[x,y]| / |[a,b]| >= c, in integers.
 *   oracle_cd32/16/8     squared Euclidean distance (Section 2.1) in float32
 *                        with a fixed summation order, see below.
 *   oracle_search_part   Alg. 1 (Graph-Search) with the POST principle of
 *                        Section 2.2 on the graph of one segment-tree node.
 *   oracle_scan_part     the linear scan of a small leaf in Alg. 4.
 *   oracle_query         Alg. 4 end to end: select, search/scan, merge.
 *   oracle_bruteforce    Def. 2.1 / Def. 2.2: exact range-filtered k-NN in
 *                        float64 (ground truth).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - Positions are 0-based ranks; the paper's [1,N] shifted by one.
 *   - Fanout f: node [a,b] of L = b-a+1 points has children
 *     j = 0..f-1 = [a + ceil(j L / f), a + ceil((j+1) L / f) - 1] (empty when
 *     the bounds cross).  At f = 2 this is Alg. 3/4's split at
 *     floor((a+b)/2).  Nodes are numbered breadth-first from the root 1;
 *     child j of node h is f (h - 1) + 2 + j (2h and 2h+1 at f = 2).
 *   - Order: every comparison uses the pair (distance, position),
 *     lexicographically, so no two candidates ever tie.
 *   - Alg. 1's stop test compares against the worst result only once Q holds
 *     m results; before that the bound is +infinity (under POST, Q may hold
 *     fewer than m points while P is not empty).
 *   - The entry point enters Q only when it lies in the query range (POST).
 *   - P holds at most cap_p candidates; inserting into a full P drops its
 *     largest entry.  cap_p >= |V| reproduces the paper's unbounded P.
 *   - Q is cut back to its m best after each expansion, as in Alg. 1.
 *   - hop_budget bounds the number of expansions (negative = unbounded).
 *   - The leaf scan scores only the part of the leaf inside the query range
 *     (the answer of Def. 2.2 lies there anyway).
 *   - Distances are squared L2.  The float32 order is: per-dimension
 *     difference rounded to float32; dimensions grouped in chunks of W
 *     consecutive values (W = 4 for float32 storage, 8 for bfloat16, 16 for
 *     fp8); G = min(64, next power of two >= number of chunks) partial sums;
 *     partial sum t takes chunks t, t+G, t+2G, ... in increasing order and
 *     inside a chunk adds each squared difference with one fused
 *     multiply-add; finally the G partial sums are added as a balanced
 *     binary tree of adjacent pairs.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -3
#define OR_EGRAPH -7

#define KIND_GRAPH 1
#define KIND_SCAN 2

#define DIST_F32 0
#define DIST_BF16 1
#define DIST_FP8 2

#define NO_NODE 0xFFFFFFFFu

/* One index as laid out in host memory (filled by the Python side from the
 * index file, with its own reader). */
typedef struct {
  int64_t n;              /* number of points */
  int32_t d;              /* dimension */
  int32_t r;              /* adjacency row width (max degree) */
  int32_t n_depth;        /* tree depths that hold at least one graph */
  int32_t leaf;           /* leaf bound: node [a,b] has a graph iff b-a >= leaf */
  int32_t c_den;          /* elastic constant c = 1/c_den */
  int32_t fanout;         /* children per tree node (chain base B of the 1-D index) */
  int32_t layout;         /* 0: segment tree (HBI-2D); 1: prefix and suffix chains (HBI-1D) */
  int32_t pad_;
  const int64_t* row_base;/* [n_depth]: row of position p in depth t is adj + (row_base[t] + p) r */
  const float* vec;       /* [n][d] float32 in position order */
  const uint16_t* vec16;  /* [n][d] bfloat16 bit patterns, or NULL */
  const uint8_t* vec8;    /* [n][d] fp8 e4m3 codes, or NULL */
  const float* scale8;    /* [n] per-vector fp8 scale, or NULL */
  const uint32_t* adj;    /* neighbour positions, NO_NODE pad (rows addressed by row_base) */
  const uint32_t* ep;     /* entry point by node number (root = 1) */
  const int64_t* ext_id;  /* [n] external id of each position */
} oracle_index;

/* ------------------------------------------------------------------------ */
/* Def. 3.1 test and Alg. 4 (subrange selection).                           */
/* ------------------------------------------------------------------------ */

/* |[x,y]| / |[a,b]| >= 1/c_den  <=>  c_den * (y-x+1) >= (b-a+1). */
int32_t oracle_elastic_ok(int64_t a, int64_t b, int64_t x, int64_t y, int32_t c_den) {
  if (!(a <= x && x <= y && y <= b)) return 0;
  return (int64_t)c_den * (y - x + 1) >= (b - a + 1);
}

/* First position of child j of the node starting at a with L points. */
static int64_t child_start(int64_t a, int64_t L, int32_t f, int64_t j) {
  return a + (j * L + f - 1) / f;
}

typedef struct {
  int64_t* out;  /* [max_parts][7]: kind, depth, heap, a, b, x, y */
  int32_t max_parts;
  int32_t n_parts;
  int64_t leaf;
  int32_t c_den;
  int32_t fanout;
} select_ctx;

static void emit_part(select_ctx* s, int64_t kind, int64_t depth, int64_t heap,
                      int64_t a, int64_t b, int64_t x, int64_t y) {
  if (s->n_parts < s->max_parts) {
    int64_t* o = s->out + 7 * (int64_t)s->n_parts;
    o[0] = kind; o[1] = depth; o[2] = heap; o[3] = a; o[4] = b; o[5] = x; o[6] = y;
  }
  s->n_parts++;
}

/* Query-2D-Index(HBI-2D, q, [a,b], [x,y]) with heap numbering of the node. */
static void query2d(select_ctx* s, int64_t a, int64_t b, int64_t depth, int64_t heap,
                    int64_t x, int64_t y) {
  /* small range: the node holds no graph, scan it */
  if (b - a < s->leaf) {
    emit_part(s, KIND_SCAN, depth, heap, a, b, x, y);
    return;
  }
  /* [x,y] inside [a,b] with ratio >= c: search this node's graph */
  if (oracle_elastic_ok(a, b, x, y, s->c_den)) {
    emit_part(s, KIND_GRAPH, depth, heap, a, b, x, y);
    return;
  }
  /* split into the f children; recurse into each one the query touches */
  int64_t L = b - a + 1;
  for (int64_t j = 0; j < s->fanout; j++) {
    int64_t ca = child_start(a, L, s->fanout, j), cb = child_start(a, L, s->fanout, j + 1) - 1;
    if (ca > cb || y < ca || x > cb) continue;
    query2d(s, ca, cb, depth + 1, (int64_t)s->fanout * (heap - 1) + 2 + j,
            x > ca ? x : ca, y < cb ? y : cb);
  }
}

/* Returns the number of parts (may exceed max_parts: only the first
 * max_parts are written), or OR_EINVAL for a bad range. */
int32_t oracle_select(int64_t n, int64_t leaf, int32_t c_den, int32_t fanout, int64_t lq,
                      int64_t rq, int64_t* parts, int32_t max_parts) {
  if (n <= 0 || leaf < 0 || c_den < 1 || fanout < 2 || lq < 0 || rq >= n || lq > rq)
    return OR_EINVAL;
  select_ctx s = {parts, max_parts, 0, leaf, c_den, fanout};
  query2d(&s, 0, n - 1, 0, 1, lq, rq);
  return s.n_parts;
}

/* Half-bounded index (Section 4.1): recorded prefixes [0, s_i - 1] with
 * s_0 = n, s_{i+1} = ceil(s_i / B) (the ranges [1, N/B^i] of Alg. 2 with
 * the division rounded up, down to one point), and the mirrored suffixes
 * [n - s_i, n - 1].  Depth i holds prefix i, depth K + i suffix i, where K
 * is the number of prefixes that own a graph (s_i - 1 >= leaf).  A query
 * [l, r] takes the tightest recorded prefix holding [0, r] -- ratio
 * (r+1)/s_i >= 1/B (Lemma 4.1) -- or, when l > 0 and r = n-1, the tightest
 * suffix holding [l, n-1].  A range with both ends inside (not
 * half-bounded; outside the index's own scope) takes whichever of the two
 * covers it with the larger ratio (ties: the prefix).  A chosen prefix or
 * suffix without a graph (s - 1 < leaf) is a linear scan of [l, r].
 * Writes one part (kind, depth, node number = depth + 1, a, b, l, r);
 * returns 1, or OR_EINVAL for a bad range. */
int64_t oracle_chain_graphs(int64_t n, int64_t leaf, int32_t base) {
  int64_t k = 0;
  for (int64_t s = n; s - 1 >= leaf; s = (s + base - 1) / base) {
    k++;
    if (s == 1) break;
  }
  return k;
}

int32_t oracle_select_1d(int64_t n, int64_t leaf, int32_t base, int64_t lq, int64_t rq,
                         int64_t* part) {
  if (n <= 0 || leaf < 0 || base < 2 || lq < 0 || rq >= n || lq > rq) return OR_EINVAL;
  int64_t K = oracle_chain_graphs(n, leaf, base);
  int64_t w = rq - lq + 1;
  /* tightest prefix holding [0, rq] and tightest suffix holding [lq, n-1] */
  int64_t sp = n, ip = 0, ss = n, is = 0;
  while (1) {
    int64_t nx = (sp + base - 1) / base;
    if (nx == sp || nx < rq + 1) break;
    sp = nx; ip++;
  }
  while (1) {
    int64_t nx = (ss + base - 1) / base;
    if (nx == ss || nx < n - lq) break;
    ss = nx; is++;
  }
  int use_prefix;
  if (lq == 0) use_prefix = 1;
  else if (rq == n - 1) use_prefix = 0;
  else use_prefix = ss >= sp;   /* w/sp >= w/ss: the prefix's ratio is at least as large */
  int64_t size = use_prefix ? sp : ss, idx = use_prefix ? ip : is;
  int64_t a = use_prefix ? 0 : n - ss, b = use_prefix ? sp - 1 : n - 1;
  (void)w;
  if (size - 1 < leaf) {        /* no graph at this size: scan the query range */
    part[0] = KIND_SCAN; part[1] = -1; part[2] = 0;
  } else {
    int64_t depth = use_prefix ? idx : K + idx;
    part[0] = KIND_GRAPH; part[1] = depth; part[2] = depth + 1;
  }
  part[3] = a; part[4] = b; part[5] = lq; part[6] = rq;
  return 1;
}

/* Elastic factor e(R,[l,r]) of Def. 3.1 over the set R of all graph nodes
 * of the fanout-f segment tree on [0,n-1]: the largest |[l,r]| / |[a,b]|
 * over recorded supersets [a,b].  Returned as the pair (num, den) of the
 * best ratio; den = 0 when no recorded node contains [l,r]. */
static void elastic_walk(int64_t a, int64_t b, int64_t leaf, int32_t f, int64_t l, int64_t r,
                         int64_t* best_num, int64_t* best_den) {
  if (b - a < leaf) return;          /* not a recorded range, nor are its children */
  if (!(a <= l && r <= b)) return;   /* not a superset */
  int64_t num = r - l + 1, den = b - a + 1;
  if (*best_den == 0 || num * (*best_den) > (*best_num) * den) {
    *best_num = num; *best_den = den;
  }
  for (int64_t j = 0; j < f; j++) {
    int64_t ca = child_start(a, den, f, j), cb = child_start(a, den, f, j + 1) - 1;
    if (ca <= cb) elastic_walk(ca, cb, leaf, f, l, r, best_num, best_den);
  }
}

int32_t oracle_elastic_factor(int64_t n, int64_t leaf, int32_t fanout, int64_t l, int64_t r,
                              int64_t* num, int64_t* den) {
  if (n <= 0 || fanout < 2 || l < 0 || r >= n || l > r) return OR_EINVAL;
  *num = 0; *den = 0;
  elastic_walk(0, n - 1, leaf, fanout, l, r, num, den);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Distances.                                                               */
/* ------------------------------------------------------------------------ */

static int32_t lanes_for(int32_t chunks) {
  int32_t g = 1;
  while (g < chunks) g *= 2;
  return g > 64 ? 64 : g;
}

/* Adjacent-pair tree over s[0..g-1] (g a power of two). */
static float pair_tree(float* s, int32_t g) {
  for (int32_t width = g; width > 1; width /= 2)
    for (int32_t i = 0; i < width / 2; i++) s[i] = s[2 * i] + s[2 * i + 1];
  return s[0];
}

/* Shared recipe: x_j supplied through a decoder. */
typedef float (*decode_fn)(const void* x, int32_t j, float scale);

static float dec_f32(const void* x, int32_t j, float scale) {
  (void)scale;
  return ((const float*)x)[j];
}

static float dec_bf16(const void* x, int32_t j, float scale) {
  (void)scale;
  uint32_t bits = (uint32_t)((const uint16_t*)x)[j] << 16;
  float f;
  memcpy(&f, &bits, 4);
  return f;
}

/* OCP 8-bit E4M3: 1 sign, 4 exponent (bias 7), 3 mantissa bits; exponent 0
 * is subnormal; code S.1111.111 is NaN; no infinities. */
float oracle_e4m3_value(uint8_t c) {
  int32_t s = c >> 7, e = (c >> 3) & 15, m = c & 7;
  float v;
  if (e == 15 && m == 7) return NAN;
  if (e == 0) v = ldexpf((float)m / 8.0f, -6);
  else v = ldexpf(1.0f + (float)m / 8.0f, e - 7);
  return s ? -v : v;
}

static float dec_fp8(const void* x, int32_t j, float scale) {
  float v = oracle_e4m3_value(((const uint8_t*)x)[j]);
  return scale * v; /* one float32 rounding */
}

static float canonical_dist(const void* x, const float* q, int32_t d, int32_t w,
                            decode_fn dec, float scale) {
  int32_t chunks = (d + w - 1) / w;
  int32_t g = lanes_for(chunks);
  float part[64];
  for (int32_t t = 0; t < g; t++) {
    float acc = 0.0f;
    for (int32_t c = t; c < chunks; c += g) {
      for (int32_t e = 0; e < w; e++) {
        int32_t j = c * w + e;
        if (j >= d) continue; /* zero padding: fma(0,0,acc) == acc */
        float delta = dec(x, j, scale) - q[j];
        acc = fmaf(delta, delta, acc);
      }
    }
    part[t] = acc;
  }
  return pair_tree(part, g);
}

float oracle_cd32(const float* x, const float* q, int32_t d) {
  return canonical_dist(x, q, d, 4, dec_f32, 1.0f);
}
float oracle_cd16(const uint16_t* x, const float* q, int32_t d) {
  return canonical_dist(x, q, d, 8, dec_bf16, 1.0f);
}
float oracle_cd8(const uint8_t* x, float scale, const float* q, int32_t d) {
  return canonical_dist(x, q, d, 16, dec_fp8, scale);
}

static float dist_of(const oracle_index* ix, int32_t kind, int64_t p, const float* q) {
  int32_t d = ix->d;
  if (kind == DIST_BF16) return oracle_cd16(ix->vec16 + p * d, q, d);
  if (kind == DIST_FP8) return oracle_cd8(ix->vec8 + p * d, ix->scale8[p], q, d);
  return oracle_cd32(ix->vec + p * d, q, d);
}

/* ------------------------------------------------------------------------ */
/* Ordered lists of (distance, position).                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
  float dist;
  int64_t pos;
} cand;

static int cand_less(cand u, cand v) {
  return u.dist < v.dist || (u.dist == v.dist && u.pos < v.pos);
}

/* Sorted ascending array with a capacity; insertion keeps the order. */
typedef struct {
  cand* a;
  int64_t len, cap;
} sorted_list;

static int list_init(sorted_list* l, int64_t cap) {
  l->a = (cand*)malloc(sizeof(cand) * (size_t)(cap > 0 ? cap : 1));
  l->len = 0;
  l->cap = cap;
  return l->a != NULL;
}

static void list_free(sorted_list* l) { free(l->a); }

static void list_insert(sorted_list* l, cand c) {
  int64_t i = l->len;
  while (i > 0 && cand_less(c, l->a[i - 1])) {
    l->a[i] = l->a[i - 1];
    i--;
  }
  l->a[i] = c;
  l->len++;
}

static cand list_pop_min(sorted_list* l) {
  cand c = l->a[0];
  memmove(l->a, l->a + 1, sizeof(cand) * (size_t)(l->len - 1));
  l->len--;
  return c;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 with POST on one graph node.                                      */
/* ------------------------------------------------------------------------ */

/* Searches the graph of the tree node [a,b] at `depth` for the points of
 * [x,y] nearest to q.  Writes the final Q (at most m entries, ascending) to
 * q_dist/q_pos, the visited points (discovery order) to `visited` when it
 * is not NULL, and the number of expansions to *hops. */
/* Learned beam width (not in the paper): when switch_hop >= 0 and the
 * search reaches switch_hop expansions and goes on (its next candidate
 * passes the stop test of Alg. 1), the features of the state are written
 * to feat (12 doubles, when not NULL) and, when ef2 > 0, P and Q keep
 * their ef2 best and the search continues with m = cap_p = ef2.  A search
 * that stops right there takes no switch.  w_query and n_parts describe
 * the whole query; k is the answer size. */
typedef struct {
  int64_t switch_hop;
  int32_t ef2;       /* > 0: new beam width */
  int32_t k;
  int64_t w_query;
  int32_t n_parts;
  int32_t pad_;
  double* feat;
  int64_t hop2;      /* > 0: at most hop2 further expansions (stopping step) */
} oracle_switch;

/* The live part of P: candidates that can still be expanded, i.e. all of
 * P while Q holds fewer than m results, else those not farther than the
 * worst of Q (the stop bound only tightens, so the others never are). */
static int64_t live_count(const sorted_list* P, const sorted_list* Q, int32_t m) {
  if (Q->len < m) return P->len;
  int64_t c = 0;
  for (int64_t i = 0; i < P->len; i++)
    if (!cand_less(Q->a[Q->len - 1], P->a[i])) c++;
  return c;
}

static void probe_features(const oracle_switch* sw, const sorted_list* P, const sorted_list* Q,
                           int32_t m, int64_t cap_p, int64_t a, int64_t b, int64_t x, int64_t y,
                           double d_ep, int64_t n_inr, int64_t nv, double* f) {
  double wp = (double)(y - x + 1), L = (double)(b - a + 1);
  int64_t kk = sw->k < Q->len ? sw->k : Q->len;
  double q0 = Q->len > 0 ? (double)Q->a[0].dist : d_ep;
  double qk = kk > 0 ? (double)Q->a[kk - 1].dist : d_ep;
  double p0 = (double)P->a[0].dist;
  double den = d_ep > 0.0 ? d_ep : 1.0;
  double fill = (double)Q->len / (double)sw->k;
  f[0] = log2(wp);
  f[1] = log2(L);
  f[2] = wp / L;
  f[3] = log2((double)sw->w_query);
  f[4] = (double)(sw->n_parts - 1);
  f[5] = (double)live_count(P, Q, m) / (double)cap_p;
  f[6] = fill < 4.0 ? fill : 4.0;
  f[7] = (double)n_inr / (double)nv;
  f[8] = q0 / den;
  f[9] = qk / den;
  f[10] = qk > 0.0 ? p0 / qk : 1.0;
  f[11] = log2(1.0 + (double)nv);
}

int32_t oracle_search_part_sw(const oracle_index* ix, int32_t depth, int64_t heap,
                              int64_t a, int64_t b, int64_t x, int64_t y, const float* q,
                              int32_t m, int64_t cap_p, int64_t hop_budget, int32_t kind,
                              float* q_dist, int64_t* q_pos, int32_t* q_len,
                              int64_t* visited, int64_t visited_cap, int64_t* n_visited,
                              int64_t* hops, const oracle_switch* sw);

int32_t oracle_search_part(const oracle_index* ix, int32_t depth, int64_t heap,
                           int64_t a, int64_t b, int64_t x, int64_t y, const float* q,
                           int32_t m, int64_t cap_p, int64_t hop_budget, int32_t kind,
                           float* q_dist, int64_t* q_pos, int32_t* q_len,
                           int64_t* visited, int64_t visited_cap, int64_t* n_visited,
                           int64_t* hops) {
  return oracle_search_part_sw(ix, depth, heap, a, b, x, y, q, m, cap_p, hop_budget, kind,
                               q_dist, q_pos, q_len, visited, visited_cap, n_visited, hops, NULL);
}

int32_t oracle_search_part_sw(const oracle_index* ix, int32_t depth, int64_t heap,
                              int64_t a, int64_t b, int64_t x, int64_t y, const float* q,
                              int32_t m, int64_t cap_p, int64_t hop_budget, int32_t kind,
                              float* q_dist, int64_t* q_pos, int32_t* q_len,
                              int64_t* visited, int64_t visited_cap, int64_t* n_visited,
                              int64_t* hops, const oracle_switch* sw) {
  if (m < 1 || cap_p < 1 || depth < 0 || depth >= ix->n_depth) return OR_EINVAL;
  if (!(0 <= a && a <= x && x <= y && y <= b && b < ix->n)) return OR_EINVAL;
  int64_t n_heap = 1, level = 1;                  /* node numbers of depths < n_depth */
  if (ix->layout == 1) n_heap = ix->n_depth + 1;  /* chains: node number = depth + 1 */
  else
    for (int32_t t = 0; t < ix->n_depth; t++) { n_heap += level; level *= ix->fanout; }
  if (heap < 1 || heap >= n_heap) return OR_EINVAL;
  uint32_t ep = ix->ep[heap];
  if (ep == NO_NODE || (int64_t)ep < a || (int64_t)ep > b) return OR_EGRAPH;
  const uint32_t* rows = ix->adj + ix->row_base[depth] * ix->r;

  int64_t span = b - a + 1;
  uint8_t* seen = (uint8_t*)calloc((size_t)span, 1); /* visited flags of [a,b] */
  sorted_list P, Q;
  if (!seen || !list_init(&P, cap_p + 1) || !list_init(&Q, (int64_t)m + ix->r + 1)) {
    free(seen);
    return OR_ENOMEM;
  }
  int64_t nv = 0, h = 0, n_inr = 0;

  /* P <- ep ; Q <- ep (POST: only if in range) */
  cand e = {dist_of(ix, kind, ep, q), ep};
  n_inr = (x <= (int64_t)ep && (int64_t)ep <= y) ? 1 : 0;
  seen[ep - a] = 1;
  if (visited && nv < visited_cap) visited[nv] = ep;
  nv++;
  list_insert(&P, e);
  if (x <= (int64_t)ep && (int64_t)ep <= y) list_insert(&Q, e);

  int32_t status = OR_OK;
  while (P.len > 0) {
    if (sw && sw->switch_hop >= 0 && h == sw->switch_hop &&
        !(Q.len >= m && cand_less(Q.a[Q.len - 1], P.a[0]))) {
      if (sw->feat)
        probe_features(sw, &P, &Q, m, cap_p, a, b, x, y, (double)e.dist, n_inr, nv, sw->feat);
      if (sw->hop2 > 0 && (hop_budget < 0 || h + sw->hop2 < hop_budget))
        hop_budget = h + sw->hop2;                     /* stopping step */
      if (sw->ef2 > 0) {                               /* keep the ef2 best of P and Q */
        if (P.len > sw->ef2) P.len = sw->ef2;
        if (Q.len > sw->ef2) Q.len = sw->ef2;
        m = sw->ef2;
        cap_p = sw->ef2;
      }
    }
    cand u = P.a[0];                                   /* u <- P.top() */
    if (Q.len >= m && cand_less(Q.a[Q.len - 1], u)) break; /* farther than worst of a full Q */
    if (hop_budget >= 0 && h >= hop_budget) break;
    list_pop_min(&P);
    h++;
    for (int32_t s = 0; s < ix->r; s++) {               /* for v in N(u) */
      uint32_t v = rows[u.pos * ix->r + s];
      if (v == NO_NODE) continue;
      if ((int64_t)v < a || (int64_t)v > b) { status = OR_EGRAPH; continue; }
      if (seen[v - a]) continue;                        /* visited */
      seen[v - a] = 1;
      if (visited && nv < visited_cap) visited[nv] = v;
      nv++;
      cand c = {dist_of(ix, kind, v, q), v};
      if (x <= (int64_t)v && (int64_t)v <= y) n_inr++;
      list_insert(&P, c);                               /* P <- P u v */
      if (P.len > cap_p) P.len = cap_p;                 /* drop the largest */
      if ((int64_t)v < x || (int64_t)v > y) continue;   /* POST: out of range */
      list_insert(&Q, c);                               /* Q <- Q u v */
    }
    if (Q.len > m) Q.len = m;                           /* keep the m best */
  }

  for (int64_t i = 0; i < Q.len; i++) {
    q_dist[i] = Q.a[i].dist;
    q_pos[i] = Q.a[i].pos;
  }
  *q_len = (int32_t)Q.len;
  *n_visited = nv;
  *hops = h;
  list_free(&P);
  list_free(&Q);
  free(seen);
  return status;
}

/* Linear scan of [x,y] (inside a leaf), top min(k, y-x+1) by (CD32, pos). */
int32_t oracle_scan_part(const oracle_index* ix, int64_t x, int64_t y, const float* q,
                         int32_t k, float* out_dist, int64_t* out_pos, int32_t* out_len) {
  if (k < 1 || x < 0 || y >= ix->n || x > y) return OR_EINVAL;
  sorted_list L;
  if (!list_init(&L, (int64_t)k + 1)) return OR_ENOMEM;
  for (int64_t p = x; p <= y; p++) {
    cand c = {oracle_cd32(ix->vec + p * ix->d, q, ix->d), p};
    list_insert(&L, c);
    if (L.len > k) L.len = k;
  }
  for (int64_t i = 0; i < L.len; i++) {
    out_dist[i] = L.a[i].dist;
    out_pos[i] = L.a[i].pos;
  }
  *out_len = (int32_t)L.len;
  list_free(&L);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Alg. 4 end to end.                                                       */
/* ------------------------------------------------------------------------ */

#define MAX_PARTS 64

/* stats (optional, 8 entries): n_parts, total hops, total visited,
 * n_graph_parts, n_scan_parts, status of the worst part, 0, 0.
 * rerank != 0 recomputes the final Q of every graph part in float32 before
 * taking its top k (used with bfloat16 / fp8 traversal). */
/* Alg. 4 with the learned beam width: graph part i switches to ef2[i]
 * after switch_hop expansions (ef2[i] <= 0: no switch for that part). */
int32_t oracle_query_sw(const oracle_index* ix, const float* q, int64_t lq, int64_t rq,
                        int32_t k, int32_t ef, int64_t cap_p, int64_t hop_budget,
                        int32_t kind, int32_t rerank, int64_t switch_hop, const int32_t* ef2,
                        const int64_t* hop2, int64_t* ids, float* dists, int64_t* stats);

int32_t oracle_query(const oracle_index* ix, const float* q, int64_t lq, int64_t rq,
                     int32_t k, int32_t ef, int64_t cap_p, int64_t hop_budget,
                     int32_t kind, int32_t rerank, int64_t* ids, float* dists,
                     int64_t* stats) {
  return oracle_query_sw(ix, q, lq, rq, k, ef, cap_p, hop_budget, kind, rerank, -1, NULL, NULL,
                         ids, dists, stats);
}

int32_t oracle_query_sw(const oracle_index* ix, const float* q, int64_t lq, int64_t rq,
                        int32_t k, int32_t ef, int64_t cap_p, int64_t hop_budget,
                        int32_t kind, int32_t rerank, int64_t switch_hop, const int32_t* ef2,
                        const int64_t* hop2, int64_t* ids, float* dists, int64_t* stats) {
  for (int32_t i = 0; i < k; i++) {
    ids[i] = -1;
    dists[i] = INFINITY;
  }
  if (stats) memset(stats, 0, sizeof(int64_t) * 8);
  if (k < 1 || ef < k) return OR_EINVAL;
  int64_t parts[MAX_PARTS * 7];
  int32_t np = ix->layout == 1
                   ? oracle_select_1d(ix->n, ix->leaf, ix->fanout, lq, rq, parts)
                   : oracle_select(ix->n, ix->leaf, ix->c_den, ix->fanout, lq, rq, parts,
                                   MAX_PARTS);
  if (np < 0) return np;
  if (np > MAX_PARTS) return OR_EINVAL;

  sorted_list M; /* merge of every part's top k */
  if (!list_init(&M, (int64_t)k * np + 1)) return OR_ENOMEM;
  float* pd = (float*)malloc(sizeof(float) * (size_t)(ef + 1));
  int64_t* pp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ef + 1));
  int32_t status = OR_OK;
  for (int32_t i = 0; i < np && pd && pp; i++) {
    const int64_t* o = parts + 7 * i;
    int32_t len = 0;
    int32_t st;
    if (o[0] == KIND_SCAN) {
      st = oracle_scan_part(ix, o[5], o[6], q, k, pd, pp, &len);
      if (stats) { stats[2] += o[6] - o[5] + 1; stats[4]++; }
    } else {
      int64_t nv = 0, h = 0;
      oracle_switch sw = {switch_hop, ef2 ? ef2[i] : 0, k, rq - lq + 1, np, 0, NULL,
                          hop2 ? hop2[i] : 0};
      st = oracle_search_part_sw(ix, (int32_t)o[1], o[2], o[3], o[4], o[5], o[6], q, ef,
                                 cap_p, hop_budget, kind, pd, pp, &len, NULL, 0, &nv, &h,
                                 (switch_hop >= 0 && (ef2 || hop2)) ? &sw : NULL);
      if (stats) { stats[1] += h; stats[2] += nv; stats[3]++; }
      if (st == OR_OK && rerank && kind != DIST_F32) {
        sorted_list R;
        if (!list_init(&R, (int64_t)len + 1)) { st = OR_ENOMEM; }
        else {
          for (int32_t j = 0; j < len; j++) {
            cand c = {oracle_cd32(ix->vec + pp[j] * ix->d, q, ix->d), pp[j]};
            list_insert(&R, c);
          }
          for (int32_t j = 0; j < len; j++) { pd[j] = R.a[j].dist; pp[j] = R.a[j].pos; }
          list_free(&R);
        }
      }
    }
    if (st != OR_OK) status = st;
    for (int32_t j = 0; j < len && j < k; j++) {
      cand c = {pd[j], pp[j]};
      list_insert(&M, c);
    }
  }
  if (!pd || !pp) status = OR_ENOMEM;
  for (int64_t i = 0; i < M.len && i < k; i++) {
    ids[i] = ix->ext_id[M.a[i].pos];
    dists[i] = M.a[i].dist;
  }
  if (stats) { stats[0] = np; stats[5] = status; }
  free(pd);
  free(pp);
  list_free(&M);
  return status;
}

/* Many queries, spread over OpenMP threads (the CPU baseline).  status[i]
 * receives each query's return code; stats is [nq][8] or NULL. */
int32_t oracle_query_batch(const oracle_index* ix, const float* qs, const int64_t* lq,
                           const int64_t* rq, int64_t nq, int32_t k, int32_t ef,
                           int64_t cap_p, int64_t hop_budget, int32_t kind, int32_t rerank,
                           int64_t* ids, float* dists, int64_t* stats, int32_t* status) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < nq; i++) {
    status[i] = oracle_query(ix, qs + i * ix->d, lq[i], rq[i], k, ef, cap_p, hop_budget,
                             kind, rerank, ids + i * k, dists + i * k,
                             stats ? stats + 8 * i : NULL);
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact range-filtered k-NN in float64 (Def. 2.1 and Def. 2.2).            */
/* ------------------------------------------------------------------------ */

typedef struct {
  double dist;
  int64_t pos;
} cand64;

static int cand64_less(cand64 u, cand64 v) {
  return u.dist < v.dist || (u.dist == v.dist && u.pos < v.pos);
}

/* vec in position order; writes min(k, rq-lq+1) positions and float64
 * distances, ascending by (distance, position). */
int32_t oracle_bruteforce(const float* vec, int64_t n, int32_t d, const float* q,
                          int64_t lq, int64_t rq, int32_t k, int64_t* out_pos,
                          double* out_dist) {
  if (k < 1 || lq < 0 || rq >= n || lq > rq) return OR_EINVAL;
  cand64* best = (cand64*)malloc(sizeof(cand64) * (size_t)(k + 1));
  if (!best) return OR_ENOMEM;
  int64_t len = 0;
  for (int64_t p = lq; p <= rq; p++) {
    double s = 0.0;
    for (int32_t j = 0; j < d; j++) {
      double t = (double)vec[p * d + j] - (double)q[j];
      s += t * t;
    }
    cand64 c = {s, p};
    if (len == k && !cand64_less(c, best[len - 1])) continue;
    int64_t i = len < k ? len++ : len - 1;
    while (i > 0 && cand64_less(c, best[i - 1])) {
      best[i] = best[i - 1];
      i--;
    }
    best[i] = c;
  }
  for (int64_t i = 0; i < k; i++) {
    out_pos[i] = i < len ? best[i].pos : -1;
    out_dist[i] = i < len ? best[i].dist : INFINITY;
  }
  free(best);
  return OR_OK;
}

int32_t oracle_bruteforce_batch(const float* vec, int64_t n, int32_t d, const float* qs,
                                const int64_t* lq, const int64_t* rq, int64_t nq, int32_t k,
                                int64_t* out_pos, double* out_dist, int32_t* status) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < nq; i++)
    status[i] = oracle_bruteforce(vec, n, d, qs + i * d, lq[i], rq[i], k, out_pos + i * k,
                                  out_dist + i * k);
  return OR_OK;
}
