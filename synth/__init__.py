"""Seeded synthetic workloads for range-filtered k-NN search.

This module only draws random numbers: it holds none of the search method's
arithmetic, so both the product path and the oracle may take their inputs
from here.  Each workload mirrors the shape of the paper's experiments
(Section 5.1: 1M-point image/text embedding sets, attribute values
synthesised independently of the vectors, ranges drawn at random or with a
fixed length that is a power-of-two fraction of N) at the sizes of the five
named workloads below.  The real datasets (SIFT, DEEP, GLOVE, WIT) are not
used; these mixtures stand in for them.

Conventions
-----------
* ``X[i]`` is point ``i`` (its external id) in the original, unsorted order.
* ``attr[i]`` is the point's numeric attribute.  Every workload uses a random
  permutation of ``0..N-1``, so attribute values coincide with attribute
  ranks (the re-ranking of the paper's footnote in Section 1 maps any
  attribute to its rank).
* A query is ``(Q[j], l[j], r[j])`` with an inclusive rank range.
* Generator streams are numpy PCG64 with seeds ``1000+c`` (data),
  ``2000+c`` (attribute permutation), ``3000+c`` (query vectors),
  ``4000+c`` (ranges) and ``5000+c`` (extra query sets, e.g. training
  traces) for workload ``c``.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

__all__ = ["Workload", "WORKLOADS", "make_workload", "fixed_width_ranges", "half_bounded_ranges",
           "spread_norms",
           "sha256_of"]


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape and law of one synthetic workload."""

    cid: int                 # workload number, selects the seeds
    name: str
    n: int                   # database size N
    d: int                   # dimension
    n_centres: int           # mixture components
    law: str                 # "gauss" | "uint8" | "unit"
    nq: int                  # number of queries
    ranges: str              # "loguniform_frac" | "buckets" | "loguniform_pts"
    range_lo: float          # lower end of the width law (fraction or points)
    n_buckets: int           # for "buckets": widths floor(N * 2^-b), b < n_buckets
    k: int
    ef: int
    leaf: int                # leaf bound: a tree node [a,b] with b-a < leaf has no graph
    degree: int = 16          # max out-degree R; 32 = the layer-0 bound of HNSW with M = 16
    ef_construction: int = 200


WORKLOADS = {
    # Tiny: 16-centre Gaussian mixture, centres N(0,4I), unit spread.
    0: Workload(0, "tiny-gauss-10k-d32", 10_000, 32, 16, "gauss", 200,
                "loguniform_frac", 0.01, 0, k=10, ef=64, leaf=128),
    # SIFT-shaped: integer values 0..255 from a clipped, rounded mixture.
    1: Workload(1, "sift-shaped-1M-d128-u8", 1_000_000, 128, 64, "uint8", 10_000,
                "buckets", 0.0, 11, k=10, ef=64, leaf=1024, degree=32),
    # DEEP-shaped batched mix: unit-norm 256-centre mixture, widths 10..N.
    2: Workload(2, "deep-shaped-1M-d96-unit", 1_000_000, 96, 256, "unit", 100_000,
                "loguniform_pts", 10.0, 0, k=10, ef=64, leaf=1024, degree=32),
    # Embedding-shaped: unit-norm 512-centre mixture in d=768.
    3: Workload(3, "embedding-shaped-2M-d768-unit", 2_000_000, 768, 512, "unit", 20_000,
                "buckets", 0.0, 13, k=100, ef=256, leaf=1024, degree=32),
}


def _centres(rng: np.random.Generator, w: Workload) -> np.ndarray:
    if w.law == "gauss":
        return (2.0 * rng.standard_normal((w.n_centres, w.d))).astype(np.float64)
    if w.law == "uint8":
        return 48.0 + 32.0 * rng.standard_normal((w.n_centres, w.d))
    if w.law == "unit":
        return rng.standard_normal((w.n_centres, w.d))
    raise ValueError(w.law)


def _draw_points(rng: np.random.Generator, w: Workload, centres: np.ndarray,
                 n: int, chunk: int = 1 << 18) -> np.ndarray:
    """Draw ``n`` mixture points in float32, chunk by chunk (bounded memory)."""
    out = np.empty((n, w.d), dtype=np.float32)
    cid = rng.integers(0, w.n_centres, size=n)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        z = rng.standard_normal((e - s, w.d), dtype=np.float32)
        c = centres[cid[s:e]].astype(np.float32)
        if w.law == "gauss":
            x = c + z
        elif w.law == "uint8":
            x = np.clip(np.rint(c + np.float32(16.0) * z), 0.0, 255.0)
        else:  # unit
            x = c + np.float32(0.5) * z
            nrm = np.sqrt(np.sum(x.astype(np.float64) ** 2, axis=1, keepdims=True))
            x = (x / nrm).astype(np.float32)
        out[s:e] = x
    return out


def _ranges(rng: np.random.Generator, w: Workload, n: int, nq: int):
    if w.ranges == "loguniform_frac":
        lo = max(1.0, w.range_lo * n)
        width = np.rint(np.exp(rng.uniform(math.log(lo), math.log(n), size=nq)))
    elif w.ranges == "loguniform_pts":
        lo = min(float(n), w.range_lo)
        width = np.rint(np.exp(rng.uniform(math.log(lo), math.log(n), size=nq)))
    elif w.ranges == "buckets":
        b = rng.permutation(np.arange(nq) % w.n_buckets)
        width = np.floor(n * np.power(2.0, -b.astype(np.float64)))
    else:
        raise ValueError(w.ranges)
    width = np.clip(width.astype(np.int64), 1, n)
    l = (rng.random(nq) * (n - width + 1)).astype(np.int64)
    l = np.minimum(l, n - width)
    r = l + width - 1
    return l, r


def make_workload(cid: int, n: int | None = None, nq: int | None = None,
                  query_stream: int = 3000, range_stream: int = 4000,
                  d: int | None = None) -> dict:
    """Generate workload ``cid``, optionally shrunk to ``n`` points / ``nq`` queries.

    Shrinking keeps every law; it only changes N (and the widths, which are
    fractions of N or capped by N).  ``query_stream``/``range_stream`` select
    the seed offsets of the query set, so a second, disjoint set (training
    traces) uses 5000.
    """
    w = WORKLOADS[cid]
    if d is not None:
        w = dataclasses.replace(w, d=d)
    n = w.n if n is None else int(n)
    nq = w.nq if nq is None else int(nq)
    rng_data = np.random.Generator(np.random.PCG64(1000 + cid))
    rng_attr = np.random.Generator(np.random.PCG64(2000 + cid))
    rng_q = np.random.Generator(np.random.PCG64(query_stream + cid))
    rng_r = np.random.Generator(np.random.PCG64(range_stream + cid))
    centres = _centres(rng_data, w)
    X = _draw_points(rng_data, w, centres, n)
    attr = rng_attr.permutation(n).astype(np.int64)
    Q = _draw_points(rng_q, w, centres, nq) if nq > 0 else np.zeros((0, w.d), np.float32)
    l, r = _ranges(rng_r, w, n, nq)
    return dict(workload=w, name=w.name, n=n, d=w.d, X=X, attr=attr, Q=Q,
                l=l, r=r, k=w.k, ef=w.ef, leaf=w.leaf, degree=w.degree,
                ef_construction=w.ef_construction)


def fixed_width_ranges(n: int, nq: int, frac: float, seed: int):
    """nq ranges of width floor(n * frac) at uniform random offsets (the
    fixed-length ranges of the paper's experiments, e.g. 2^-5 N)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    width = max(1, int(math.floor(n * frac)))
    l = (rng.random(nq) * (n - width + 1)).astype(np.int64)
    l = np.minimum(l, n - width)
    return l, l + width - 1


def half_bounded_ranges(n: int, nq: int, lo: float, seed: int):
    """nq half-bounded ranges: even queries are prefixes [0, w-1], odd ones
    suffixes [n-w, n-1], widths log-uniform over [lo, n] points (the
    half-bounded queries of the paper's Section 4.1 and Exp-1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = min(float(n), float(lo))
    width = np.clip(np.rint(np.exp(rng.uniform(math.log(lo), math.log(n), size=nq))), 1, n)
    width = width.astype(np.int64)
    pre = np.arange(nq) % 2 == 0
    l = np.where(pre, 0, n - width).astype(np.int64)
    r = np.where(pre, width - 1, n - 1).astype(np.int64)
    return l, r


def spread_norms(X: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """Rows of X rescaled by exp(sigma z), z standard normal per row: the
    log-normal spread of norms of inner-product workloads (for instance
    recommendation embeddings), where the largest inner product and the
    nearest point differ."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = np.exp(sigma * rng.standard_normal(X.shape[0]))
    return (X.astype(np.float64) * s[:, None]).astype(np.float32)


def sha256_of(*arrays: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()
