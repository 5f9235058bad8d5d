"""CPU oracle for ESG range-filtered k-NN search -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the bench
may import this package.  It shares no code with the product (the HIP
library and its Python binding): it reads index files with its own reader,
encodes bfloat16 / fp8 with its own encoders written from the format
definitions, and runs the plain C routines of ``esg_oracle.c``.

Contents and the passage each follows:

* ``read_index``          -- own reader of the documented index file layout.
* ``select``              -- Alg. 4 subrange selection (Section 4.2).
* ``select_1d``           -- the half-bounded index's query rule (Section
                             4.1, Lemma 4.1).
* ``elastic_factor``      -- Def. 3.1 over the recorded ranges of the tree.
* ``cd32/cd16/cd8``       -- squared Euclidean distance (Section 2.1) in
                             float32 with the fixed summation order.
* ``search_part``         -- Alg. 1 + POST (Sections 2.1, 2.2) on one node.
* ``query/query_batch``   -- Alg. 4 end to end (select, search/scan, merge).
* ``bruteforce``          -- Def. 2.1 / 2.2 exact filtered k-NN in float64.
* ``recall``              -- recall@k against exact ground truth, counting a
                             returned point as correct when its exact
                             distance does not exceed the k-th true one.
* ``bf16_encode`` / ``e4m3_encode`` -- storage codecs (round to nearest
                             even; fp8 OCP E4M3 with a per-vector scale).
* ``mlp_*``               -- float64 forward and manual backward of the
                             12-64-64-1 ReLU network that predicts ef.
* ``adam_step64``         -- one Adam step (Kingma and Ba, Algorithm 1) in
                             float64.
* ``metric_store64``      -- the vectors an angular or inner-product index
                             stores (unit rows; the Euclidean transform of
                             Bachrach et al. 2014), in float64.
* ``exact_metric``        -- exact filtered top-k by Euclidean distance,
                             cosine similarity or inner product, in float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import struct

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "esg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KIND_GRAPH, KIND_SCAN = 1, 2
DIST_F32, DIST_BF16, DIST_FP8 = 0, 1, 2
METRIC_L2, METRIC_ANGULAR, METRIC_IP = 0, 1, 2   # the index file's metric field
NO_NODE = 0xFFFFFFFF


def compile_oracle(force: bool = False) -> str:
    """Compile esg_oracle.c into liboracle.so (no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = f"{_LIB}.{os.getpid()}.tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # ESG_ORACLE_LIB points the tests' mutation checks at a deliberately
        # broken copy of the oracle.
        path = os.environ.get("ESG_ORACLE_LIB") or compile_oracle()
        _lib = ctypes.CDLL(path)
        _declare(_lib)
    return _lib


class _Index(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("r", ctypes.c_int32),
                ("n_depth", ctypes.c_int32), ("leaf", ctypes.c_int32), ("c_den", ctypes.c_int32),
                ("fanout", ctypes.c_int32), ("layout", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("row_base", ctypes.c_void_p),
                ("vec", ctypes.c_void_p), ("vec16", ctypes.c_void_p), ("vec8", ctypes.c_void_p),
                ("scale8", ctypes.c_void_p), ("adj", ctypes.c_void_p), ("ep", ctypes.c_void_p),
                ("ext_id", ctypes.c_void_p)]


def _declare(L):
    i64, i32, vp, f32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_float
    L.oracle_select.argtypes = [i64, i64, i32, i32, i64, i64, vp, i32]
    L.oracle_select.restype = i32
    L.oracle_elastic_ok.argtypes = [i64, i64, i64, i64, i32]
    L.oracle_elastic_ok.restype = i32
    L.oracle_elastic_factor.argtypes = [i64, i64, i32, i64, i64, vp, vp]
    L.oracle_select_1d.argtypes = [i64, i64, i32, i64, i64, vp]
    L.oracle_select_1d.restype = i32
    L.oracle_chain_graphs.argtypes = [i64, i64, i32]
    L.oracle_chain_graphs.restype = i64
    L.oracle_elastic_factor.restype = i32
    L.oracle_cd32.argtypes = [vp, vp, i32]
    L.oracle_cd32.restype = f32
    L.oracle_cd16.argtypes = [vp, vp, i32]
    L.oracle_cd16.restype = f32
    L.oracle_cd8.argtypes = [vp, f32, vp, i32]
    L.oracle_cd8.restype = f32
    L.oracle_e4m3_value.argtypes = [ctypes.c_uint8]
    L.oracle_e4m3_value.restype = f32
    L.oracle_search_part.argtypes = [vp, i32, i64, i64, i64, i64, i64, vp, i32, i64, i64, i32,
                                     vp, vp, vp, vp, i64, vp, vp]
    L.oracle_search_part.restype = i32
    L.oracle_search_part_sw.argtypes = [vp, i32, i64, i64, i64, i64, i64, vp, i32, i64, i64,
                                        i32, vp, vp, vp, vp, i64, vp, vp, vp]
    L.oracle_search_part_sw.restype = i32
    L.oracle_query_sw.argtypes = [vp, vp, i64, i64, i32, i32, i64, i64, i32, i32, i64, vp, vp,
                                  vp, vp, vp]
    L.oracle_query_sw.restype = i32
    L.oracle_scan_part.argtypes = [vp, i64, i64, vp, i32, vp, vp, vp]
    L.oracle_scan_part.restype = i32
    L.oracle_query.argtypes = [vp, vp, i64, i64, i32, i32, i64, i64, i32, i32, vp, vp, vp]
    L.oracle_query.restype = i32
    L.oracle_query_batch.argtypes = [vp, vp, vp, vp, i64, i32, i32, i64, i64, i32, i32,
                                     vp, vp, vp, vp]
    L.oracle_query_batch.restype = i32
    L.oracle_bruteforce.argtypes = [vp, i64, i32, vp, i64, i64, i32, vp, vp]
    L.oracle_bruteforce.restype = i32
    L.oracle_bruteforce_batch.argtypes = [vp, i64, i32, vp, vp, vp, i64, i32, vp, vp, vp]
    L.oracle_bruteforce_batch.restype = i32


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Index file reader (layout documented with the C ABI, version 1).
# --------------------------------------------------------------------------

class OracleIndex:
    """Arrays of one index in host memory plus the C view the oracle uses."""

    def __init__(self, n, d, degree, leaf, n_depth, c_den, ext_id, attr, vec, adj, ep, fanout=2,
                 layout=0, row_base=None, metric=METRIC_L2, dq=None, max_norm2=0.0):
        self.n, self.d, self.degree, self.leaf = int(n), int(d), int(degree), int(leaf)
        # metric the stored vectors were made from; a query row holds dq values
        self.metric, self.max_norm2 = int(metric), float(max_norm2)
        self.dq = self.d if dq is None else int(dq)
        self.n_depth, self.c_den, self.fanout = int(n_depth), int(c_den), int(fanout)
        self.layout = int(layout)
        # row of position p at depth t: adj_flat[(row_base[t] + p) * degree]
        self.row_base = (np.arange(self.n_depth, dtype=np.int64) * self.n if row_base is None
                         else np.ascontiguousarray(row_base, dtype=np.int64))
        self.ext_id = np.ascontiguousarray(ext_id, dtype=np.int64)
        self.attr = np.ascontiguousarray(attr, dtype=np.float64)
        self.vec = np.ascontiguousarray(vec, dtype=np.float32)
        self.adj = np.ascontiguousarray(adj, dtype=np.uint32)
        self.ep = np.ascontiguousarray(ep, dtype=np.uint32)
        self.vec16 = None
        self.vec8 = None
        self.scale8 = None
        self._c = None

    def select(self, lq: int, rq: int):
        """Alg. 4 on this index's tree (its leaf bound, fanout and c), or the
        half-bounded index's rule for a chain index."""
        if self.layout == 1:
            return select_1d(self.n, self.leaf, int(lq), int(rq), base=self.fanout)
        return select(self.n, self.leaf, int(lq), int(rq), c_den=self.c_den, fanout=self.fanout)

    def stored_query(self, q) -> np.ndarray:
        """A query as the search reads it: its dq values, then zeros up to
        the stored length d (the inner-product transform's last coordinate
        of a query is 0)."""
        q = np.asarray(q, np.float32)
        if q.shape[-1] == self.d:
            return np.ascontiguousarray(q)
        if q.shape[-1] != self.dq:
            raise ValueError("query length")
        out = np.zeros(q.shape[:-1] + (self.d,), np.float32)
        out[..., :self.dq] = q
        return out

    def rows(self, depth: int):
        """Adjacency rows of a depth, indexed by position (a view)."""
        flat = self.adj.reshape(-1, self.degree)
        return flat[self.row_base[depth]:]

    def with_bf16(self):
        self.vec16 = bf16_encode(self.vec)
        self._c = None
        return self

    def with_fp8(self):
        self.vec8, self.scale8 = e4m3_encode_rows(self.vec)
        self._c = None
        return self

    def cstruct(self):
        if self._c is None:
            s = _Index()
            s.n, s.d, s.r, s.n_depth = self.n, self.d, self.degree, self.n_depth
            s.leaf, s.c_den, s.fanout = self.leaf, self.c_den, self.fanout
            s.layout, s.pad_, s.row_base = self.layout, 0, _p(self.row_base)
            s.vec, s.vec16, s.vec8 = _p(self.vec), _p(self.vec16), _p(self.vec8)
            s.scale8, s.adj, s.ep, s.ext_id = _p(self.scale8), _p(self.adj), _p(self.ep), _p(self.ext_id)
            self._c = s
        return ctypes.byref(self._c)


def read_index(path: str) -> OracleIndex:
    with open(path, "rb") as f:
        head = f.read(144)
    if len(head) < 144 or head[:8] != b"ESGIDX01":
        raise ValueError("not an index file")
    version, header_bytes = struct.unpack_from("<II", head, 8)
    n, = struct.unpack_from("<q", head, 16)
    d, degree, leaf, fanout, n_depth, c_den, efc, layout = struct.unpack_from("<8i", head, 24)
    off_ids, off_attr, off_vec, off_adj, off_ep, file_bytes = struct.unpack_from("<6Q", head, 56)
    metric, dq = struct.unpack_from("<2i", head, 124)
    max_norm2, = struct.unpack_from("<d", head, 132)
    if version != 2 or fanout < 2:
        raise ValueError("unsupported index version/fanout")
    mkw = dict(metric=metric, dq=dq, max_norm2=max_norm2)
    mm = np.memmap(path, dtype=np.uint8, mode="r")
    if mm.size != file_bytes:
        raise ValueError("truncated index file")

    def sect(off, dtype, count):
        return np.frombuffer(mm, dtype=dtype, count=count, offset=off)

    ext_id = sect(off_ids, np.int64, n)
    attr = sect(off_attr, np.float64, n)
    vec = sect(off_vec, np.float32, n * d).reshape(n, d)
    if layout == 1:
        sizes, starts = chain_levels(n, leaf, fanout)
        assert len(sizes) == n_depth
        row_base = np.cumsum([0] + sizes[:-1]) - np.array(starts, np.int64)
        adj = sect(off_adj, np.uint32, int(sum(sizes)) * degree)
        ep = sect(off_ep, np.uint32, n_depth + 1)
        return OracleIndex(n, d, degree, leaf, n_depth, c_den, ext_id, attr, vec, adj, ep, fanout,
                           layout=1, row_base=row_base, **mkw)
    adj = sect(off_adj, np.uint32, n_depth * n * degree).reshape(n_depth, n, degree)
    ep = sect(off_ep, np.uint32, node_numbers(fanout, n_depth))
    return OracleIndex(n, d, degree, leaf, n_depth, c_den, ext_id, attr, vec, adj, ep, fanout,
                       **mkw)


def chain_levels(n: int, leaf: int, base: int):
    """Depths of the half-bounded index: the recorded prefixes [0, s_i - 1]
    that own a graph (s_0 = n, s_{i+1} = ceil(s_i / base), s_i - 1 >= leaf),
    then the suffixes [n - s_i, n - 1] of the same sizes.  Returns (sizes,
    first positions) per depth."""
    k = int(lib().oracle_chain_graphs(n, leaf, base))
    sizes, s = [], n
    for _ in range(k):
        sizes.append(s)
        s = -(-s // base)
    return sizes + sizes, [0] * k + [n - x for x in sizes]


def node_numbers(fanout: int, n_depth: int) -> int:
    """Length of the entry-point table: node numbers 1 .. sum of fanout^t
    over the depths t < n_depth (breadth-first from the root 1), plus the
    unused 0."""
    return 1 + sum(fanout ** t for t in range(n_depth))


# --------------------------------------------------------------------------
# Codecs, written from the format definitions.
# --------------------------------------------------------------------------

def bf16_encode(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns, round to nearest, ties to even.

    Written from the definition: the two bfloat16 values that bracket x are
    the truncation t (drop the low 16 bits) and the next one up in
    magnitude; pick the nearer in exact (float64) arithmetic and, on a tie,
    the one whose last kept bit is 0.  Inputs are finite."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    bits = x.view(np.uint32)
    lo = (bits & np.uint32(0xFFFF0000))
    hi = lo + np.uint32(0x10000)
    vlo = lo.view(np.float32).astype(np.float64)
    vhi = hi.view(np.float32).astype(np.float64)
    xv = x.astype(np.float64)
    dlo = np.abs(xv - vlo)
    dhi = np.abs(vhi - xv)
    lo_even = ((lo >> np.uint32(16)) & np.uint32(1)) == 0
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ~lo_even)
    out = np.where(pick_hi, hi, lo) >> np.uint32(16)
    return out.astype(np.uint16)


def bf16_decode(h: np.ndarray) -> np.ndarray:
    return (h.astype(np.uint32) << np.uint32(16)).view(np.float32)


def _e4m3_table() -> np.ndarray:
    L = lib()
    return np.array([L.oracle_e4m3_value(c) for c in range(256)], dtype=np.float32)


_E4M3 = None


def e4m3_values() -> np.ndarray:
    global _E4M3
    if _E4M3 is None:
        _E4M3 = _e4m3_table()
    return _E4M3


def e4m3_encode(y: np.ndarray) -> np.ndarray:
    """float32 -> OCP E4M3 codes: nearest representable value, ties to the
    code with an even mantissa, magnitudes beyond 448 saturate to +-448.
    Brute force over the 126 finite non-negative magnitudes."""
    y = np.asarray(y, dtype=np.float32)
    vals = e4m3_values()
    mags = vals[:127].astype(np.float64)          # codes 0..126: 0 .. 448 ascending
    a = np.minimum(np.abs(y.astype(np.float64)), 448.0)
    i = np.searchsorted(mags, a, side="left")      # mags[i-1] < a <= mags[i]
    i = np.clip(i, 1, 126)
    below, above = mags[i - 1], mags[i]
    d_lo, d_hi = a - below, above - a
    take_hi = (d_hi < d_lo) | ((d_hi == d_lo) & ((i & 1) == 0))
    code = np.where(take_hi, i, i - 1)
    code = np.where(a == 0.0, 0, code)
    sign = (np.signbit(y) & (code != 0)).astype(np.uint8) << 7
    return (code.astype(np.uint8) | sign)


def e4m3_encode_rows(x: np.ndarray):
    """Per-vector scale sigma = max|x| / 448 (float32; 1 for a zero vector),
    codes = e4m3(x / sigma) with the division in float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    amax = np.max(np.abs(x), axis=1)
    scale = (amax / np.float32(448.0)).astype(np.float32)
    scale = np.where(scale > 0, scale, np.float32(1.0)).astype(np.float32)
    y = (x / scale[:, None]).astype(np.float32)
    return e4m3_encode(y), scale


# --------------------------------------------------------------------------
# Wrappers.
# --------------------------------------------------------------------------

def select(n: int, leaf: int, lq: int, rq: int, c_den: int = 2, max_parts: int = 64,
           fanout: int = 2):
    """Alg. 4 parts as a list of dicts (kind, depth, heap, a, b, x, y) for a
    tree of the given fanout (elastic constant c = 1/c_den)."""
    buf = np.zeros((max_parts, 7), dtype=np.int64)
    cnt = lib().oracle_select(n, leaf, c_den, fanout, lq, rq, _p(buf), max_parts)
    if cnt < 0:
        raise ValueError(f"invalid range [{lq},{rq}] for n={n}")
    keys = ("kind", "depth", "heap", "a", "b", "x", "y")
    return [dict(zip(keys, map(int, buf[i]))) for i in range(min(cnt, max_parts))], cnt


def select_1d(n: int, leaf: int, lq: int, rq: int, base: int = 2):
    """The half-bounded index's part for [lq, rq] (one part, as a list of
    one dict like ``select``) and the count 1."""
    buf = np.zeros(7, dtype=np.int64)
    cnt = lib().oracle_select_1d(n, leaf, base, lq, rq, _p(buf))
    if cnt < 0:
        raise ValueError(f"invalid range [{lq},{rq}] for n={n}")
    keys = ("kind", "depth", "heap", "a", "b", "x", "y")
    return [dict(zip(keys, map(int, buf)))], 1


def elastic_factor(n: int, leaf: int, l: int, r: int, fanout: int = 2):
    num = np.zeros(1, np.int64)
    den = np.zeros(1, np.int64)
    st = lib().oracle_elastic_factor(n, leaf, fanout, l, r, _p(num), _p(den))
    if st != 0:
        raise ValueError("bad range")
    return int(num[0]), int(den[0])


def cd32(x: np.ndarray, q: np.ndarray) -> np.float32:
    x = np.ascontiguousarray(x, np.float32)
    q = np.ascontiguousarray(q, np.float32)
    return np.float32(lib().oracle_cd32(_p(x), _p(q), x.size))


def cd16(xh: np.ndarray, q: np.ndarray) -> np.float32:
    xh = np.ascontiguousarray(xh, np.uint16)
    q = np.ascontiguousarray(q, np.float32)
    return np.float32(lib().oracle_cd16(_p(xh), _p(q), xh.size))


def cd8(codes: np.ndarray, scale: float, q: np.ndarray) -> np.float32:
    codes = np.ascontiguousarray(codes, np.uint8)
    q = np.ascontiguousarray(q, np.float32)
    return np.float32(lib().oracle_cd8(_p(codes), float(scale), _p(q), codes.size))


def search_part(ix: OracleIndex, part: dict, q: np.ndarray, m: int, cap_p: int | None = None,
                hop_budget: int = -1, kind: int = DIST_F32, visited_cap: int = 1 << 22):
    """Alg. 1 + POST on the node of ``part``.  Returns (dists, positions,
    visited (discovery order), hops, status)."""
    q = ix.stored_query(q)
    cap_p = m if cap_p is None else cap_p
    qd = np.zeros(m, np.float32)
    qp = np.zeros(m, np.int64)
    ql = np.zeros(1, np.int32)
    vis = np.zeros(visited_cap, np.int64)
    nv = np.zeros(1, np.int64)
    hops = np.zeros(1, np.int64)
    st = lib().oracle_search_part(ix.cstruct(), part["depth"], part["heap"], part["a"], part["b"],
                                  part["x"], part["y"], _p(q), m, cap_p, hop_budget, kind,
                                  _p(qd), _p(qp), _p(ql), _p(vis), visited_cap, _p(nv), _p(hops))
    L = int(ql[0])
    return qd[:L], qp[:L], vis[:min(int(nv[0]), visited_cap)], int(hops[0]), st


class _Switch(ctypes.Structure):
    _fields_ = [("switch_hop", ctypes.c_int64), ("ef2", ctypes.c_int32), ("k", ctypes.c_int32),
                ("w_query", ctypes.c_int64), ("n_parts", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("feat", ctypes.c_void_p), ("hop2", ctypes.c_int64)]


def search_part_learned(ix: OracleIndex, part: dict, q, ef_max: int, switch_hop: int, ef2: int,
                        k: int, w_query: int, n_parts: int, kind: int = DIST_F32,
                        visited_cap: int = 1 << 22):
    """Alg. 1 + POST with the learned switch: after switch_hop expansions
    at m = cap = ef_max, keep the ef2 best of P and Q and continue with
    m = cap = ef2 (ef2 <= 0: features only).  Returns (dists, positions,
    visited, hops, status, float64 features (12) or None)."""
    q = ix.stored_query(q)
    qd = np.zeros(ef_max, np.float32)
    qp = np.zeros(ef_max, np.int64)
    ql = np.zeros(1, np.int32)
    vis = np.zeros(visited_cap, np.int64)
    nv = np.zeros(1, np.int64)
    hops = np.zeros(1, np.int64)
    feat = np.full(12, np.nan)
    sw = _Switch(switch_hop, ef2, k, w_query, n_parts, 0, feat.ctypes.data, 0)
    st = lib().oracle_search_part_sw(ix.cstruct(), part["depth"], part["heap"], part["a"],
                                     part["b"], part["x"], part["y"], _p(q), ef_max, ef_max, -1,
                                     kind, _p(qd), _p(qp), _p(ql), _p(vis), visited_cap, _p(nv),
                                     _p(hops), ctypes.byref(sw))
    L = int(ql[0])
    return (qd[:L], qp[:L], vis[:min(int(nv[0]), visited_cap)], int(hops[0]), st,
            None if np.isnan(feat[0]) else feat)


def query_learned(ix: OracleIndex, q, lq, rq, k, ef_max, switch_hop, ef2_parts, kind=DIST_F32,
                  rerank=0, hop2_parts=None):
    """Alg. 4 where graph part i switches to ef2_parts[i] after switch_hop
    expansions (the beam widths a predictor chose), or, with hop2_parts,
    stops after hop2_parts[i] further expansions (the stopping steps)."""
    q = ix.stored_query(q)
    ids = np.zeros(k, np.int64)
    dists = np.zeros(k, np.float32)
    stats = np.zeros(8, np.int64)
    e2 = np.ascontiguousarray(ef2_parts, np.int32)
    h2 = None if hop2_parts is None else np.ascontiguousarray(hop2_parts, np.int64)
    st = lib().oracle_query_sw(ix.cstruct(), _p(q), lq, rq, k, ef_max, ef_max, -1, kind, rerank,
                               switch_hop, _p(e2), _p(h2), _p(ids), _p(dists), _p(stats))
    return ids, dists, stats, st


def query(ix: OracleIndex, q, lq, rq, k, ef, cap_p=None, hop_budget=-1, kind=DIST_F32, rerank=0):
    q = ix.stored_query(q)
    ids = np.zeros(k, np.int64)
    dists = np.zeros(k, np.float32)
    stats = np.zeros(8, np.int64)
    st = lib().oracle_query(ix.cstruct(), _p(q), lq, rq, k, ef, ef if cap_p is None else cap_p,
                            hop_budget, kind, rerank, _p(ids), _p(dists), _p(stats))
    return ids, dists, stats, st


def query_batch(ix: OracleIndex, Q, l, r, k, ef, cap_p=None, hop_budget=-1, kind=DIST_F32,
                rerank=0, with_stats=False):
    Q = ix.stored_query(Q)
    l = np.ascontiguousarray(l, np.int64)
    r = np.ascontiguousarray(r, np.int64)
    nq = Q.shape[0]
    ids = np.zeros((nq, k), np.int64)
    dists = np.zeros((nq, k), np.float32)
    stats = np.zeros((nq, 8), np.int64) if with_stats else None
    status = np.zeros(nq, np.int32)
    lib().oracle_query_batch(ix.cstruct(), _p(Q), _p(l), _p(r), nq, k, ef,
                             ef if cap_p is None else cap_p, hop_budget, kind, rerank,
                             _p(ids), _p(dists), _p(stats), _p(status))
    return (ids, dists, status, stats) if with_stats else (ids, dists, status)


def bruteforce(vec_pos: np.ndarray, Q, l, r, k):
    """Exact filtered k-NN (float64) over position-ordered vectors.
    Returns (positions [nq,k] (-1 pad), float64 distances [nq,k] (+inf pad))."""
    vec_pos = np.ascontiguousarray(vec_pos, np.float32)
    Q = np.ascontiguousarray(np.atleast_2d(Q), np.float32)
    l = np.ascontiguousarray(np.atleast_1d(l), np.int64)
    r = np.ascontiguousarray(np.atleast_1d(r), np.int64)
    nq = Q.shape[0]
    pos = np.zeros((nq, k), np.int64)
    dist = np.zeros((nq, k), np.float64)
    status = np.zeros(nq, np.int32)
    n, d = vec_pos.shape
    lib().oracle_bruteforce_batch(_p(vec_pos), n, d, _p(Q), _p(l), _p(r), nq, k,
                                  _p(pos), _p(dist), _p(status))
    if np.any(status != 0):
        raise ValueError("invalid range in bruteforce")
    return pos, dist


def exact_dist64(vec_pos: np.ndarray, q: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """float64 squared distances of the given positions (-1 -> +inf)."""
    pos = np.asarray(pos)
    out = np.full(pos.shape, np.inf)
    ok = pos >= 0
    diff = vec_pos[pos[ok]].astype(np.float64) - np.asarray(q, np.float64)
    out[ok] = np.sum(diff * diff, axis=-1)
    return out


def recall(vec_pos, Q, l, r, pos_found, gt_pos, gt_dist, k):
    """Mean recall@k.  A returned position counts when it lies in [l,r] and
    its float64 distance is <= the k-th exact distance (ties are credited);
    the count is divided by min(k, r-l+1).  Also returns the strict
    id-overlap recall."""
    nq = Q.shape[0]
    rec = np.zeros(nq)
    strict = np.zeros(nq)
    for i in range(nq):
        w = int(r[i] - l[i] + 1)
        kk = min(k, w)
        found = pos_found[i][pos_found[i] >= 0]
        found = found[(found >= l[i]) & (found <= r[i])]
        found = np.unique(found)
        # both sides through the same float64 routine, so equal points compare equal
        dk = exact_dist64(vec_pos, Q[i], gt_pos[i][kk - 1:kk])[0]
        df = exact_dist64(vec_pos, Q[i], found)
        rec[i] = min(kk, int(np.sum(df <= dk))) / kk
        strict[i] = len(np.intersect1d(found, gt_pos[i][:kk])) / kk
    return float(rec.mean()), float(strict.mean()), rec


# --------------------------------------------------------------------------
# Other metrics.  The paper states the method for Euclidean distance and
# names inner product and angular distance as open (Section 7); the index
# reduces them to Euclidean distance over transformed vectors.
# --------------------------------------------------------------------------

def metric_store64(X, metric: int):
    """The vectors an index of the given metric stores, in float64, and M^2.

    Angular: every row scaled to unit norm; then |x - q|^2 = 1 + |q|^2 -
    2 |q| cos(x, q), so increasing distance is decreasing cosine.  Inner
    product: the one-coordinate transform of Bachrach et al. (RecSys 2014),
    x' = [x, sqrt(M^2 - |x|^2)] with M^2 the largest squared norm, and a
    query q' = [q, 0]; then |x' - q'|^2 = M^2 + |q|^2 - 2 <x, q>."""
    X = np.asarray(X, np.float64)
    n2 = np.sum(X * X, axis=1)
    if metric == METRIC_L2:
        return X.copy(), 0.0
    if metric == METRIC_ANGULAR:
        return X / np.sqrt(n2)[:, None], 0.0
    if metric == METRIC_IP:
        m2 = float(n2.max())
        return np.hstack([X, np.sqrt(np.maximum(m2 - n2, 0.0))[:, None]]), m2
    raise ValueError("metric")


def exact_metric(X_pos, Q, l, r, k: int, metric: int):
    """Exact range-filtered top-k under a metric, from its definition, in
    float64 over the original vectors in position order: squared Euclidean
    distance increasing, cosine similarity decreasing, or inner product
    decreasing; ties by position.  Returns (positions [nq,k], -1 pad;
    scores [nq,k] float64: the distance, cosine or inner product; nan pad)."""
    X = np.asarray(X_pos, np.float64)
    Q = np.atleast_2d(np.asarray(Q, np.float64))
    l, r = np.atleast_1d(l), np.atleast_1d(r)
    nq = Q.shape[0]
    pos = np.full((nq, k), -1, np.int64)
    score = np.full((nq, k), np.nan)
    for i in range(nq):
        a, b = int(l[i]), int(r[i])
        seg, q = X[a:b + 1], Q[i]
        if metric == METRIC_L2:
            s = np.sum((seg - q) ** 2, axis=1)
            key = s
        elif metric == METRIC_ANGULAR:
            s = (seg @ q) / (np.sqrt(np.sum(seg * seg, axis=1)) * np.sqrt(q @ q))
            key = -s
        elif metric == METRIC_IP:
            s = seg @ q
            key = -s
        else:
            raise ValueError("metric")
        order = np.lexsort((np.arange(len(seg)), key))[:k]
        pos[i, :len(order)] = a + order
        score[i, :len(order)] = s[order]
    return pos, score


# --------------------------------------------------------------------------
# Beam-width predictor in float64 (forward and manual backward).
# --------------------------------------------------------------------------
# Parameter vector layout: W1[64][12] b1[64] W2[64][64] b2[64] W3[64] b3[1]
# mean[12] scale[12]; loss = mean over samples of (y - t)^2.

MLP_SIZES = [("W1", (64, 12)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64,)),
             ("b3", (1,)), ("mu", (12,)), ("sd", (12,))]


def mlp_unpack(params):
    out, o = {}, 0
    p = np.asarray(params, np.float64)
    for name, shape in MLP_SIZES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def mlp_forward64(params, F):
    P = mlp_unpack(params)
    X = (np.asarray(F, np.float64) - P["mu"]) / P["sd"]
    A1 = X @ P["W1"].T + P["b1"]
    H1 = np.maximum(A1, 0.0)
    A2 = H1 @ P["W2"].T + P["b2"]
    H2 = np.maximum(A2, 0.0)
    return H2 @ P["W3"] + P["b3"][0], (X, A1, H1, A2, H2)


def mlp_grad64(params, F, T):
    """Gradient of mean (y - t)^2 w.r.t. the 5,057 trainable weights, by the
    chain rule written out layer by layer; returns (grad, loss)."""
    P = mlp_unpack(params)
    y, (X, A1, H1, A2, H2) = mlp_forward64(params, F)
    B = len(y)
    err = y - np.asarray(T, np.float64)
    gy = 2.0 * err / B                         # dL/dy
    gW3 = gy @ H2
    gb3 = np.array([gy.sum()])
    gA2 = np.outer(gy, P["W3"]) * (A2 > 0)    # dL/da2
    gW2 = gA2.T @ H1
    gb2 = gA2.sum(0)
    gA1 = (gA2 @ P["W2"]) * (A1 > 0)          # dL/da1
    gW1 = gA1.T @ X
    gb1 = gA1.sum(0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, gb3])
    return grad, float(np.mean(err ** 2))


# --------------------------------------------------------------------------
# Adam (Kingma and Ba, "Adam: A Method for Stochastic Optimization",
# Algorithm 1) in float64.  The decay rates and epsilon are the float32
# numbers nearest 0.9, 0.999 and 1e-8 (the optimizer's constants are float32
# values); everything else is float64.
# --------------------------------------------------------------------------

ADAM_B1 = float(np.float32(0.9))
ADAM_B2 = float(np.float32(0.999))
ADAM_EPS = float(np.float32(1e-8))


def adam_step64(theta, g, m, v, t, lr):
    """Step t (>= 1): biased first and second moment estimates, their bias
    corrections by 1 - beta^t, and the update theta - lr * mhat /
    (sqrt(vhat) + eps).  Returns (theta, m, v) as new float64 arrays."""
    theta, g = np.asarray(theta, np.float64), np.asarray(g, np.float64)
    m, v = np.asarray(m, np.float64), np.asarray(v, np.float64)
    m = ADAM_B1 * m + (1.0 - ADAM_B1) * g
    v = ADAM_B2 * v + (1.0 - ADAM_B2) * g * g
    mhat = m / (1.0 - ADAM_B1 ** t)
    vhat = v / (1.0 - ADAM_B2 ** t)
    return theta - float(lr) * mhat / (np.sqrt(vhat) + ADAM_EPS), m, v
