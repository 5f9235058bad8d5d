/*
 * esg.h -- C ABI of libesg, an MI355X (gfx950) engine for range-filtered
 * approximate k-nearest-neighbour search with elastic graphs (ESG,
 * Yang et al.).
 *
 * Problem (Def. 2.2): the database holds N vectors in R^d, each with a
 * numeric attribute.  Points are re-ranked by attribute (footnote of
 * Section 1), so a point's attribute rank is its *position* p in [0, N-1]
 * (the paper's [1,N], shifted to 0-based).  A query (q, l, r) asks for the
 * (approximate) k points nearest to q in Euclidean distance (Def. 2.1)
 * among the positions l <= p <= r.
 *
 * Index (Section 4.2, HBI-2D): a segment tree of fanout f over [0, N-1]
 * (f = 2 in Alg. 3/4; larger f is the extension of Section 4.2).  Node
 * [a,b] of L points has children j = 0..f-1 = [a + ceil(jL/f),
 * a + ceil((j+1)L/f) - 1] (at f = 2: split at floor((a+b)/2)); a node with
 * b - a >= leaf holds a proximity graph over its points (Alg. 3); smaller
 * nodes are scanned.  A query picks at most two nodes (Alg. 4, Lemma 4.2,
 * Lemma 4.3) whose graphs cover [l,r] with ratio |part| / |node| >= 1/f
 * (Def. 3.1 with the elastic constant c = 1/f), searches each with
 * Alg. 1 under the POST principle (Section 2.2) -- out-of-range points are
 * traversed but never returned -- and merges the two answers.
 *
 * Conventions for every entry point:
 *  - Return value 0 (ESG_OK) or a negative ESG_E* code; nothing throws or
 *    aborts across this boundary.  esg_status_str() names the code.
 *  - "device" pointers are HIP device memory on the index's device; "host"
 *    pointers are ordinary CPU memory.  The caller owns every buffer it
 *    passes; the library owns the memory behind an esg_index.
 *  - Distances are squared Euclidean distances in float32.
 *  - All ordering uses the pair (distance, position): ties never occur.
 *  - An esg_index may be used by one stream at a time.
 */
#ifndef ESG_H_
#define ESG_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define ESG_OK 0
#define ESG_EINVAL (-1)      /* bad argument (null pointer, size, k/ef)     */
#define ESG_ERANGE (-2)      /* value out of the supported range            */
#define ESG_ENOMEM (-3)      /* host or device allocation failed            */
#define ESG_EIO (-4)         /* file could not be opened / read / written   */
#define ESG_EFORMAT (-5)     /* index file malformed or checksum mismatch   */
#define ESG_EHIP (-6)        /* a HIP runtime call failed                   */
#define ESG_EUNSUPPORTED (-7)/* feature not available for this index       */
#define ESG_EOVERFLOW (-8)   /* a bounded device structure overflowed       */

#define ESG_EF_MAX 1024      /* largest beam width m (= ef) accepted        */
#define ESG_DEGREE_MAX 32    /* largest graph degree accepted               */
#define ESG_FANOUT_MAX 64    /* largest segment-tree fanout accepted        */
#define ESG_NO_NODE 0xFFFFFFFFu /* padding value of an adjacency row        */

/* ---- index file (version 2), little-endian ------------------------------
 * bytes [0,512): header
 *   char     magic[8]  = "ESGIDX01"
 *   uint32   version   = 2, header_bytes = 512
 *   int64    n;  int32 d, degree, leaf, fanout, n_depth, c_den, ef_construction, layout
 *   uint64   off_ids, off_attr, off_vec, off_adj, off_ep, file_bytes
 *   uint32   crc32c of the sections ids, attr, vec, adj, ep (in that order)
 *   int32    metric, dq;  float64 max_norm2   (see ESG_METRIC_*)
 *   uint32   crc32c of header bytes [0,140)
 * sections (each 4096-aligned):
 *   ids  int64  [n]                external id of the point at position p
 *   attr float64[n]                sorted attribute values (rank -> value)
 *   vec  float32[n][d]             vectors in position order
 *   adj  uint32 [n_depth][n][degree]  row p of depth t: neighbours of p in
 *                                  the graph of the depth-t node holding p,
 *                                  positions inside that node, ESG_NO_NODE pad
 *   ep   uint32 [1 + sum_{t<n_depth} fanout^t]  entry point of the tree
 *                                  node numbered h: root 1, child j of node h
 *                                  numbered fanout*(h-1) + 2 + j (2h, 2h+1 at
 *                                  fanout 2); ESG_NO_NODE where the node has
 *                                  no graph
 * c_den is the elastic constant's denominator (c = 1/c_den); the builder
 * writes c_den = fanout and the loader requires c_den >= fanout.
 * layout 1 (half-bounded index, Section 4.1): the recorded sizes are
 *   s_0 = n, s_{i+1} = ceil(s_i / fanout) while s_i - 1 >= leaf (K of them);
 *   n_depth = 2K; depth i < K is the graph of the prefix [0, s_i - 1] and
 *   depth K + i that of the suffix [n - s_i, n - 1]; adj holds each depth's
 *   rows for its own positions only, depth after depth (2 sum s_i rows);
 *   ep is uint32 [n_depth + 1], the entry of depth t at index t + 1.
 *   A query takes the tightest prefix holding [0, r] (Lemma 4.1: ratio
 *   >= 1/fanout), or for l > 0 and r = n-1 the tightest suffix holding
 *   [l, n-1]; a range with both ends inside takes whichever of the two has
 *   the larger ratio (the prefix on a tie); one that needs a size without a
 *   graph is scanned.
 * ----------------------------------------------------------------------- */

/* Metrics.  Every index searches by squared Euclidean distance over its
 * stored vectors; the other metrics are reduced to it when the index is
 * built (the paper states its method for Euclidean space and leaves other
 * metrics open, Section 7):
 *   ESG_METRIC_L2       stored = input; dq = d.
 *   ESG_METRIC_ANGULAR  stored = input / |input| (float64 norm, rounded to
 *       float32); dq = d.  For a query q the distance is 1 + |q|^2 - 2 cos
 *       (x, q) |q|, so the order is that of decreasing cosine similarity.
 *   ESG_METRIC_IP       maximum inner product by the one-coordinate
 *       Euclidean transform of Bachrach et al. (RecSys 2014): with
 *       M^2 = max |x|^2, stored x' = [x, sqrt(M^2 - |x|^2)] (d = input d + 1)
 *       and a query of dq = d - 1 values is read as [q, 0], so
 *       |x' - q'|^2 = M^2 + |q|^2 - 2 <x, q>: increasing distance is
 *       decreasing inner product, and <x, q> = (M^2 + |q|^2 - dist) / 2.
 * Search calls take queries of dq float32 values per row and return the
 * stored-space squared distance. */
#define ESG_METRIC_L2 0
#define ESG_METRIC_ANGULAR 1
#define ESG_METRIC_IP 2

typedef struct {
  int32_t degree;          /* max out-degree R of every graph (<= 32), 16   */
  int32_t leaf;            /* leaf bound: node [a,b] has a graph iff b-a >= leaf (>= 1) */
  int32_t ef_construction; /* beam width of the insertion searches, 200     */
  int32_t fanout;          /* segment-tree fanout f in [2, ESG_FANOUT_MAX]
                              (0 = 2); the elastic constant is c = 1/f    */
  int32_t threads;         /* host threads, 0 = all                         */
  int32_t batch_max;       /* largest insertion batch, 0 = default (1024)   */
  int32_t verbose;         /* print progress to stderr                      */
  int32_t layout;          /* 0: segment tree (HBI-2D, Section 4.2); 1: the
                              half-bounded index (HBI-1D, Section 4.1):
                              prefix and suffix chains with base = fanout */
  int32_t metric;          /* ESG_METRIC_L2 (0), _ANGULAR or _IP            */
} esg_build_params;

/* Builds the HBI-2D index of Alg. 3 on the host and writes it to out_path.
 * vecs: host float32 [n][d] row-major, point i = external id i; d is the
 *       input length (the stored length is d + 1 for ESG_METRIC_IP).
 * attr: host float64 [n] attribute values (any order; equal values are
 *       ranked by external id).  The library ranks them itself, so
 *       positions are attribute ranks (ties by external id).
 * Each internal node's graph is a copy of its first child's graph plus the
 * insertion of its other points (Alg. 3; at fanout 2 the right half); a
 * node whose first child is a leaf first builds that child's points from
 * scratch.  Insertion is a beam search of
 * width ef_construction followed by occlusion pruning (Section 2.1) to at
 * most `degree` neighbours and reverse edges.  Points are inserted in
 * deterministic batches, so the file does not depend on `threads`.
 * Errors: EINVAL (null/size, unknown metric, a zero or non-finite vector
 * under ESG_METRIC_ANGULAR, a non-finite norm under ESG_METRIC_IP),
 * EUNSUPPORTED (fanout > ESG_FANOUT_MAX), ERANGE (tree too deep), ENOMEM,
 * EIO. */
int32_t esg_build_index(const float* vecs, const double* attr, int64_t n, int32_t d,
                        const esg_build_params* params, const char* out_path);

/* The same build with the insertion rounds on HIP device `hip_device`: for
 * each round (the batches of every node of one depth, inserted against the
 * graphs as they were before the round), the beam searches run in the
 * search kernel, and the occlusion pruning and the reverse edges (grouped
 * per target) in kernels of their own; distances use the float32
 * summation order of the search kernels on both paths.  Entry points
 * (medoids in float64) and the reachability repair stay on the host
 * between depths.  Writes the same file as esg_build_index for the same
 * inputs and parameters.  Needs batch_max <= 8192 and a dimension with
 * compiled kernels.  Device memory: the vectors (4 n d bytes), every
 * depth's rows (4 n R n_depth), the search workspace of a loaded index,
 * and buffers for rounds of up to 65,536 points.
 * Errors: those of esg_build_index, plus EUNSUPPORTED (dimension),
 * EHIP. */
int32_t esg_build_index_gpu(const float* vecs, const double* attr, int64_t n, int32_t d,
                            const esg_build_params* params, int32_t hip_device,
                            const char* out_path);

/* ---- loaded index -------------------------------------------------------- */
typedef struct esg_index esg_index;

typedef struct {
  int64_t n;
  int32_t d, degree, leaf, fanout, n_depth, c_den;
  int32_t has_bf16, has_fp8;  /* device copies made by esg_index_add_storage */
  int64_t device_bytes;       /* device memory owned by the index           */
  int32_t metric, dq;         /* ESG_METRIC_*; values per query row         */
  double max_norm2;           /* ESG_METRIC_IP: M^2; else 0                 */
} esg_index_info_t;

/* Reads the index file, checks magic, sizes and checksums, and copies it to
 * HIP device `hip_device` (plus the fixed search workspace).  On success
 * *out owns all of it until esg_free_index.  Kernels are compiled for the
 * stored lengths 32, 64, 96, 128, 256, 512, 768, 1024 and 2048; each serves
 * every length with the same number of lanes per vector and chunks per
 * lane, which covers d = 17 .. 1024 and 1793 .. 2048.  Errors: EINVAL,
 * EIO, EFORMAT, ENOMEM, EHIP, EUNSUPPORTED (a length no kernel serves). */
int32_t esg_load_index(const char* path, int32_t hip_device, esg_index** out);

/* Adds a reduced-precision traversal copy of the vectors on the device:
 * kind 1 = bfloat16 (round to nearest even), kind 2 = fp8 OCP e4m3 with a
 * per-vector float32 scale max|x|/448 (saturating, nearest-even).  The
 * float32 copy stays for the rerank.  stream: hipStream_t or NULL. */
int32_t esg_index_add_storage(esg_index* idx, int32_t kind, void* stream);

/* Copies the device vectors of `kind` (0 float32 [n][d], 1 bfloat16 bits
 * [n][d], 2 fp8 codes [n][d] followed by float32 scales [n]) to host memory
 * `dst` of `bytes` bytes (must be exactly the size listed).  Synchronous.
 * For inspection and tests.  Errors: EINVAL (size), EUNSUPPORTED (no such
 * copy), EHIP. */
int32_t esg_index_copy_storage(const esg_index* idx, int32_t kind, void* dst, int64_t bytes);

int32_t esg_index_info(const esg_index* idx, esg_index_info_t* out);
void esg_free_index(esg_index* idx);
const char* esg_status_str(int32_t status);

/* ---- search --------------------------------------------------------------
 * queries: device float32 [nq][d] row-major
 * l, r:    device int64 [nq], inclusive position range; a query with
 *          l < 0, r > N-1 or l > r is invalid: its output row is all -1 /
 *          +inf and it is counted in n_invalid (opts), the batch goes on.
 * k, ef:   1 <= k <= ef <= ESG_EF_MAX; ef is the beam width m of Alg. 1.
 * ids:     device int64 [nq][k] out, external ids, -1 where fewer than k
 *          points lie in the range.
 * dists:   device float32 [nq][k] out, squared L2, +inf padding.
 * stream:  hipStream_t (NULL = default stream).  The call is asynchronous
 *          with respect to the host; it never allocates memory.
 * Errors (nothing launched): EINVAL, ERANGE (nq beyond the workspace),
 * EHIP.  */
int32_t esg_search_batch(esg_index* idx, const float* queries, const int64_t* l,
                         const int64_t* r, int64_t nq, int32_t k, int32_t ef,
                         int64_t* ids, float* dists, void* stream);

#define ESG_TRAV_F32 0
#define ESG_TRAV_BF16 1
#define ESG_TRAV_FP8 2

/* Optional per-part debug record (device memory, [nq][2] records). */
typedef struct {
  int32_t kind;       /* 0 none, 1 graph search, 2 leaf scan */
  int32_t depth;
  int64_t heap;       /* heap number of the tree node */
  int64_t a, b;       /* node range */
  int64_t x, y;       /* part of the query range inside the node */
  int64_t hops;       /* expansions of Alg. 1 */
  int64_t n_visited;  /* points whose distance was computed */
  int64_t ticks;      /* device wall-clock ticks (100 MHz) spent on the part */
} esg_part_trace;

typedef struct {
  int32_t traversal;     /* ESG_TRAV_*                                     */
  int32_t rerank;        /* recompute final candidates in float32           */
  int32_t cand_cap;      /* capacity of P (0 = ef)                          */
  int32_t hash_cap;      /* 16-bit LDS visited slots per wave, a power of two
                            in [64, 16384] (0 = 4096) with
                            ceil(log2 N) - log2(hash_cap) <= 12 (else
                            ERANGE); keys that find no free slot within 8
                            probes go to a global bitmap: always exact    */
  int64_t hop_budget;    /* max expansions per graph part, < 0 = unbounded  */
  int64_t router_threshold; /* > 0: queries narrower than this many positions
                            take the MFMA brute-force scan (exact, see
                            esg_scan_batch); needs bfloat16 storage and a
                            reservation (esg_index_reserve) of >= nq queries
                            and windows                                   */
  int32_t use_graph;     /* 1: capture the launch sequence in a hipGraph on
                            first use and replay it while the arguments stay
                            the same                                       */
  int32_t scan_rerank;   /* candidates recomputed in float32 by the scan
                            (0 = default, as rerank_count below)          */
  const float* mlp;      /* device ESG_MLP_PARAMS floats, or NULL: the
                            learned beam width.  Each graph part runs
                            probe_hops expansions of Alg. 1 with m = ef
                            (the largest beam); if its search goes on
                            (the next candidate passes the stop test),
                            the network maps 12 features of the search
                            state to y and the part
                            continues with m = cand_cap = ef' =
                            clamp(ceil(2^(y + mlp_delta)), k, ef), keeping
                            the ef' best of P and Q.  Layout as for
                            esg_mlp_forward; each call copies the weights
                            into the index's own inference layout on the
                            call's stream first (read-only here)          */
  int32_t probe_hops;    /* with mlp (or with feat_out alone: features
                            only, no change of beam): > 0 as above (1
                            selects a kernel whose switch comes before its
                            search loop); 0: the beam of every graph part
                            is chosen before the search from its selection
                            features alone (log2 of its filter width and
                            node size, their ratio, log2 of the query
                            width, parts - 1; the seven probe-state
                            features are 0), then the plain kernel runs
                            each part with m = cand_cap = ef'; needs a
                            reservation of >= nq queries and
                            mlp_target = 0                                */
  float mlp_delta;       /* calibration offset added to y                   */
  int32_t mlp_target;    /* 0: y sets the beam width as above; 1: y sets the
                            stopping step instead -- the part may take at
                            most ceil(2^(y + mlp_delta)) (>= 1) further
                            expansions, m stays ef                        */
  float* feat_out;       /* device float [nq][2][16] or NULL: per graph part
                            the 12 features, y and ef' (or the granted
                            expansions when mlp_target = 1) (parts that end
                            before or right at the end of the probe, and
                            leaf scans, are left untouched)               */
  esg_part_trace* trace; /* device [nq][2] or NULL                          */
  uint32_t* visited;     /* device [nq][2][visited_cap] or NULL: visited positions */
  int64_t visited_cap;   /* capacity per part of `visited`                  */
  int64_t* n_invalid;    /* device int64[1] or NULL: += invalid queries     */
  const int32_t* part_ef;/* device int32 [nq][2] or NULL: the beam of each
                            graph part (slot = the part's order), chosen by
                            the caller (for instance from feat_out of an
                            earlier call with probe_hops = 0); each part
                            runs with m = cand_cap = clamp(value, k, ef);
                            excludes mlp                                  */
} esg_search_opts;

/* Reserves the device workspace of the brute-force scan and the router:
 * per-query lists for up to max_queries queries per call and per-window
 * records for up to max_windows windows of at most 2,048 positions (about
 * 540 bytes per window).  A window's candidate list takes 64E slots of the
 * 64 reserved per window (E = 1, 2, 4 for k <= 32, 64, 128), so a call
 * handles max_windows / E windows at once: esg_scan_batch splits larger
 * batches into several passes, the router returns ERANGE.  Also holds the
 * per-part beams of the learned form without a probe (probe_hops = 0).
 * Allocates; call it once before searching.  Errors: EINVAL, ENOMEM. */
int32_t esg_index_reserve(esg_index* idx, int64_t max_queries, int64_t max_windows);

typedef struct {
  int32_t rerank_count;  /* candidates recomputed in float32 per query
                            (0 = 64E - 1, the whole merged list: the most
                            queries certified, the fewest exact rescans) */
  int32_t flags;         /* bit 0 (ESG_SCAN_EXACT): skip the certificate and
                            rescan every query exactly; other bits 0     */
  int32_t* certified;    /* device int32 [nq] out (1 = certified), or NULL */
  int64_t* n_fallback;   /* host int64 out: queries rescanned exactly, or NULL */
} esg_scan_opts;

#define ESG_SCAN_EXACT 1

/* Exact range-filtered k-NN by brute force (Def. 2.1 / 2.2 with the float32
 * canonical distance, ties by position), for any range widths: candidates
 * from bfloat16 MFMA dot products (v_mfma_f32_16x16x32_bf16, float32
 * accumulation) over windows of <= 2,048 positions, float32 rerank, and a
 * certificate from the rounding-error bound; queries that are not
 * certified are rescanned exactly.  The result equals a float32 scan of
 * [l,r].  Same buffers as esg_search_batch; k <= 128.  Copies l and r to
 * the host to plan the windows and synchronizes `stream` before returning.
 * Needs bfloat16 storage and a reservation, and stored rows of at most
 * 1,024 values.  Errors: EINVAL, EUNSUPPORTED, ERANGE, EHIP. */
int32_t esg_scan_batch(esg_index* idx, const esg_scan_opts* opts, const float* queries,
                       const int64_t* l, const int64_t* r, int64_t nq, int32_t k,
                       int64_t* ids, float* dists, void* stream);

/* ---- beam-width predictor (learned ef) ------------------------------------
 * A 12 -> 64 -> 64 -> 1 ReLU network in float32.  Parameters (device
 * float[ESG_MLP_PARAMS]): W1[64][12] b1[64] W2[64][64] b2[64] W3[64] b3[1]
 * (ESG_MLP_WEIGHTS trainable values), then the feature mean[12] and
 * scale[12] used to normalise inputs.  Features (float[n][12]) as written
 * by feat_out.  Not part of the paper; the training targets come from the
 * search's own traces (see the Python binding). */
#define ESG_MLP_FEATURES 12
#define ESG_MLP_WEIGHTS 5057
#define ESG_MLP_PARAMS 5081
#define ESG_MLP_WORKSPACE_FLOATS (512 * 5058)

/* out[i] = network(feats[i]) for i < n.  Device pointers; asynchronous. */
int32_t esg_mlp_forward(const float* params, const float* feats, int64_t n, float* out,
                        void* stream);
/* grad[ESG_MLP_WEIGHTS] = d/dw of mean_i (network(feats[i]) - target[i])^2
 * and *loss = that mean (device, may be NULL); workspace: device float
 * [ESG_MLP_WORKSPACE_FLOATS], owned by the caller.  Deterministic. */
int32_t esg_mlp_grad(const float* params, const float* feats, const float* target, int64_t n,
                     float* grad, float* loss, float* workspace, void* stream);
/* esg_mlp_grad without the caller's workspace, for callers that cannot
 * allocate device memory (code under hipGraph capture, serving loops,
 * harnesses that forbid hipMalloc).  The per-wave partial gradients go to
 * a fixed scratch array inside the library (ESG_MLP_WORKSPACE_FLOATS floats,
 * about 10 MB per GPU, held until the process ends); the call allocates
 * nothing.  Any n >= 1 fits (the scratch size does not depend on n).  All
 * calls on one GPU share that GPU's scratch: calls that overlap in time on
 * one GPU (two streams, two threads) race and must be serialised by the
 * caller.  Same results as esg_mlp_grad, bit for bit.  Errors: EINVAL,
 * EHIP. */
int32_t esg_mlp_grad_noalloc(const float* params, const float* feats, const float* target,
                             int64_t n, float* grad, float* loss, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the trainable
 * weights; m1, m2: device float[ESG_MLP_WEIGHTS] moments, step >= 1. */
int32_t esg_mlp_adam(float* params, const float* grad, float* m1, float* m2, int64_t step,
                     float lr, void* stream);

/* esg_search_batch with options; opts == NULL behaves like esg_search_batch. */
int32_t esg_search_batch_ex(esg_index* idx, const esg_search_opts* opts,
                            const float* queries, const int64_t* l, const int64_t* r,
                            int64_t nq, int32_t k, int32_t ef, int64_t* ids, float* dists,
                            void* stream);

#ifdef __cplusplus
}
#endif
#endif /* ESG_H_ */
