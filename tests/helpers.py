"""Test-side helpers: small hand-checkable trees and graphs built in numpy.

These build index arrays for the oracle directly (no product code): the
segment tree of Section 4.2 enumerated breadth-first, and per node a graph
whose rows hold the node's chain neighbours (p-1, p+1, which keeps every
node graph connected) followed by nearest neighbours in float64."""
from __future__ import annotations

import numpy as np

import oracle

NO = 0xFFFFFFFF


def tree_nodes(n: int, leaf: int, fanout: int = 2):
    """All tree nodes as (depth, heap, a, b, is_graph), breadth-first.  Node
    [a,b] of L points splits into fanout children of L/fanout points each,
    rounded so that child j starts at a + ceil(j L / fanout) (at fanout 2:
    [a, floor((a+b)/2)] and the rest); child j of node h is numbered
    fanout (h - 1) + 2 + j."""
    out = []
    todo = [(0, 1, 0, n - 1)]
    while todo:
        nxt = []
        for depth, heap, a, b in todo:
            g = (b - a) >= leaf
            out.append((depth, heap, a, b, g))
            if g and a < b:
                L = b - a + 1
                starts = [a + -(-j * L // fanout) for j in range(fanout + 1)]
                for j in range(fanout):
                    if starts[j] <= starts[j + 1] - 1:
                        nxt.append((depth + 1, fanout * (heap - 1) + 2 + j, starts[j],
                                    starts[j + 1] - 1))
        todo = nxt
    return out


def make_test_index(X: np.ndarray, leaf: int, R: int = 8, ep_mode: str = "first",
                    rng: np.random.Generator | None = None) -> oracle.OracleIndex:
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    nodes = tree_nodes(n, leaf)
    n_depth = max([t for t, _, _, _, g in nodes if g], default=-1) + 1
    adj = np.full((max(n_depth, 0), n, R), NO, dtype=np.uint32)
    ep = np.full(1 << max(n_depth, 0), NO, dtype=np.uint32)
    X64 = X.astype(np.float64)
    for t, h, a, b, g in nodes:
        if not g:
            continue
        idx = np.arange(a, b + 1)
        D = ((X64[idx, None, :] - X64[None, idx, :]) ** 2).sum(-1)
        for i, p in enumerate(idx):
            row = []
            if p - 1 >= a:
                row.append(p - 1)
            if p + 1 <= b:
                row.append(p + 1)
            order = np.lexsort((idx, D[i]))
            for j in order:
                q = idx[j]
                if len(row) >= R:
                    break
                if q != p and q not in row:
                    row.append(q)
            adj[t, p, :len(row)] = row
        if ep_mode == "first":
            ep[h] = a
        else:
            ep[h] = (rng or np.random.default_rng(h)).integers(a, b + 1)
    ext = np.arange(n, dtype=np.int64)
    return oracle.OracleIndex(n, d, R, leaf, n_depth, 2, ext, np.arange(n, dtype=np.float64),
                              X, adj, ep)


def oracle_scan(oix, Q, l, r, k):
    """The oracle's float32 linear scan of each query's whole range [l,r]
    (top k by the canonical distance, ties by position): the exact answer
    the brute-force scan must return.  Invalid ranges give -1 / +inf rows."""
    ids = np.full((len(Q), k), -1, np.int64)
    dists = np.full((len(Q), k), np.inf, np.float32)
    L = oracle.lib()
    for i in range(len(Q)):
        if l[i] < 0 or r[i] >= oix.n or l[i] > r[i]:
            continue
        od = np.zeros(k, np.float32)
        op = np.zeros(k, np.int64)
        ol = np.zeros(1, np.int32)
        q = oix.stored_query(Q[i])
        st = L.oracle_scan_part(oix.cstruct(), int(l[i]), int(r[i]), q.ctypes.data, k,
                                od.ctypes.data, op.ctypes.data, ol.ctypes.data)
        assert st == 0
        n = int(ol[0])
        ids[i, :n] = oix.ext_id[op[:n]]
        dists[i, :n] = od[:n]
    return ids, dists
