"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values
worked by hand from the paper's algorithms (tests/golden), closed forms,
lemmas, special cases that reduce to brute force or to a library routine,
and exact-arithmetic cases.  test_oracle_mutations.py plants plausible
mistakes in a copy of the oracle and checks that these pins catch them.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import oracle
from tests.helpers import make_test_index, tree_nodes

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- selector

def _parse_parts(spec: str):
    out = []
    for tok in spec.split():
        k, depth, heap, a, b, x, y = tok.split(":")
        out.append(dict(kind=oracle.KIND_GRAPH if k == "G" else oracle.KIND_SCAN,
                        depth=int(depth), heap=int(heap), a=int(a), b=int(b), x=int(x), y=int(y)))
    return out


def test_selector_golden_cases():
    """Alg. 4 on small trees, worked by hand (tests/golden/selector_cases.txt)."""
    n_cases = 0
    for line in open(os.path.join(GOLD, "selector_cases.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        lhs, rhs = line.split("|")
        n, leaf, l, r = map(int, lhs.split())
        parts, cnt = oracle.select(n, leaf, l, r)
        assert cnt == len(parts)
        assert parts == _parse_parts(rhs), (n, leaf, l, r, parts)
        n_cases += 1
    assert n_cases >= 10


def test_selector_fanout_golden_cases():
    """Alg. 4 on fanout-4 trees with c = 1/4 (Section 4.2, Extensions),
    worked by hand (tests/golden/selector_cases_fanout.txt)."""
    n_cases = 0
    for line in open(os.path.join(GOLD, "selector_cases_fanout.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        lhs, rhs = line.split("|")
        n, leaf, f, l, r = map(int, lhs.split())
        parts, cnt = oracle.select(n, leaf, l, r, c_den=f, fanout=f)
        assert cnt == len(parts)
        assert parts == _parse_parts(rhs), (n, leaf, f, l, r, parts)
        n_cases += 1
    assert n_cases >= 14


@pytest.mark.parametrize("n,leaf,f", [(1, 1, 2), (2, 1, 2), (7, 1, 2), (16, 1, 2), (33, 2, 2),
                                      (50, 3, 2), (64, 5, 2), (89, 1, 2), (100, 16, 2),
                                      (128, 4, 2), (60, 1, 3), (90, 2, 3), (64, 1, 4),
                                      (100, 1, 4), (77, 3, 4), (130, 1, 8), (99, 2, 8),
                                      (200, 1, 16), (150, 3, 16)])
def test_selector_enumeration(n, leaf, f):
    """Every range [l,r]: at most two parts (Lemma 4.2 at fanout 2, Lemma 4.3
    at fanout f with c = 1/f); the parts tile the range left to right; each
    part lies in a tree node of the fanout-f segment tree; graph parts hold
    at least 1/f of their node (Def. 3.1) and sit on nodes that own a graph
    (Alg. 3); scans sit on leaves; a split query becomes a suffix of one
    node and a prefix of another (two half-bounded queries, Section 4.2,
    Extensions)."""
    nodes = {(h): (t, a, b, g) for t, h, a, b, g in tree_nodes(n, leaf, f)}
    for l in range(n):
        for r in range(l, n):
            parts, cnt = oracle.select(n, leaf, l, r, c_den=f, fanout=f)
            assert 1 <= cnt <= 2
            cur = l
            for p in parts:
                t, a, b, g = nodes[p["heap"]]
                assert (p["depth"], p["a"], p["b"]) == (t, a, b)
                assert a <= p["x"] <= p["y"] <= b
                assert p["x"] == cur
                cur = p["y"] + 1
                if p["kind"] == oracle.KIND_GRAPH:
                    assert g and f * (p["y"] - p["x"] + 1) >= b - a + 1
                else:
                    assert b - a < leaf
            assert cur == r + 1
            if cnt == 2:
                assert parts[0]["y"] == parts[0]["b"] and parts[1]["x"] == parts[1]["a"]


def test_fanout_lemma_needs_c_at_most_one_over_f():
    """Lemma 4.3 ties the elastic constant to the fanout: with c = 1/2 on a
    fanout-4 tree (a stricter test than 1/4), some ranges need more than
    two parts -- so the two-part bound is the lemma's, not an accident."""
    worst = 0
    for l in range(64):
        for r in range(l, 64):
            worst = max(worst, oracle.select(64, 1, l, r, c_den=2, fanout=4)[1])
    assert worst > 2


def test_selector_1d_golden_cases():
    """The half-bounded index's query rule (Section 4.1, Lemma 4.1) worked by
    hand (tests/golden/selector_cases_1d.txt)."""
    n_cases = 0
    for line in open(os.path.join(GOLD, "selector_cases_1d.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        lhs, rhs = line.split("|")
        n, leaf, B, l, r = map(int, lhs.split())
        parts, cnt = oracle.select_1d(n, leaf, l, r, base=B)
        assert cnt == 1 and parts == _parse_parts(rhs), (n, leaf, B, l, r, parts)
        n_cases += 1
    assert n_cases >= 17


def _recorded_sizes(n, B):
    s, out = n, [n]
    while s > 1:
        s = -(-s // B)
        out.append(s)
    return out


@pytest.mark.parametrize("n,leaf,B", [(1, 1, 2), (2, 1, 2), (37, 1, 2), (100, 4, 2), (257, 8, 2),
                                      (90, 2, 3), (200, 5, 4), (500, 16, 8)])
def test_selector_1d_half_bounded(n, leaf, B):
    """Lemma 4.1 by enumeration: every prefix [0, r] and suffix [l, n-1] gets
    one recorded range holding it -- the smallest recorded one (no smaller
    recorded size holds it) -- whose ratio is >= 1/B when it owns a graph;
    a range whose tightest recorded size has no graph is scanned."""
    sizes = _recorded_sizes(n, B)
    K = sum(1 for s in sizes if s - 1 >= leaf)
    for r in range(n):
        for (l, rr, pre) in ((0, r, True), (r, n - 1, False)):
            if not pre and l == 0:
                continue
            (p,), cnt = oracle.select_1d(n, leaf, l, rr, base=B)
            w = rr - l + 1
            tight = min(s for s in sizes if s >= w)
            assert (p["x"], p["y"]) == (l, rr)
            assert (p["a"], p["b"]) == ((0, tight - 1) if pre else (n - tight, n - 1))
            if tight - 1 >= leaf:
                i = sizes.index(tight)
                assert p["kind"] == oracle.KIND_GRAPH and B * w >= tight
                assert p["depth"] == (i if pre else K + i) and p["heap"] == p["depth"] + 1
            else:
                assert p["kind"] == oracle.KIND_SCAN


def test_selector_1d_general_ranges_take_the_better_side():
    """A range with both ends inside (outside the half-bounded index's own
    scope) takes the tighter cover of the two sides (larger ratio; the
    prefix on a tie), still one part holding it."""
    n, leaf, B = 300, 4, 2
    sizes = _recorded_sizes(n, B)
    for l in range(1, n - 1, 7):
        for r in range(l, n - 1, 5):
            (p,), _ = oracle.select_1d(n, leaf, l, r, base=B)
            sp = min(s for s in sizes if s >= r + 1)
            ss = min(s for s in sizes if s >= n - l)
            want = (0, sp - 1) if ss >= sp else (n - ss, n - 1)
            assert (p["a"], p["b"]) == want and p["a"] <= l and r <= p["b"]


@pytest.mark.parametrize("n,leaf,f", [(50, 1, 2), (100, 3, 2), (1000, 16, 2), (4096, 64, 2),
                                      (100, 1, 4), (1000, 16, 8), (4096, 64, 16)])
def test_selector_half_bounded_one_part(n, leaf, f):
    """Lemma 4.1: a prefix [0,r] (or suffix) is answered by one recorded
    range holding it with ratio >= 1/f -- one part, never a split."""
    for r in range(n):
        for (l, rr) in ((0, r), (r, n - 1)):
            parts, cnt = oracle.select(n, leaf, l, rr, c_den=f, fanout=f)
            assert cnt == 1
            p = parts[0]
            if p["kind"] == oracle.KIND_GRAPH:
                assert f * (p["y"] - p["x"] + 1) >= p["b"] - p["a"] + 1


@pytest.mark.parametrize("n,leaf,f", [(20, 1, 2), (37, 2, 2), (64, 4, 2), (50, 1, 4), (70, 2, 8)])
def test_elastic_factor_definition(n, leaf, f):
    """Def. 3.1: e(R,[l,r]) is the best ratio over recorded supersets.
    Brute force over the recorded ranges R of the tree; and a graph part
    chosen by Alg. 4 never has a ratio below 1/f."""
    R = [(a, b) for _, _, a, b, g in tree_nodes(n, leaf, f) if g]
    for l in range(n):
        for r in range(l, n):
            best = None
            for a, b in R:
                if a <= l and r <= b:
                    fr = (r - l + 1) / (b - a + 1)
                    best = fr if best is None else max(best, fr)
            num, den = oracle.elastic_factor(n, leaf, l, r, fanout=f)
            if best is None:
                assert den == 0
            else:
                assert den > 0 and math.isclose(num / den, best)


# ---------------------------------------------------------------- distances

def _case_vectors(c):
    d = c["d"]
    q = np.zeros(d, np.float32)
    if "q" in c:
        q[:len(c["q"])] = c["q"]
    if c["kind"] == "fp8":
        codes = np.full(d, c["code_fill"], np.uint8)
        codes[:len(c["codes"])] = c["codes"]
        return codes, q
    x = np.full(d, c["fill"], np.float32)
    x[:len(c["x"])] = c["x"]
    return x, q


def test_distance_golden_cases():
    cases = json.load(open(os.path.join(GOLD, "distance_cases.json")))["cases"]
    for c in cases:
        x, q = _case_vectors(c)
        if c["kind"] == "f32":
            got = oracle.cd32(x, q)
        elif c["kind"] == "bf16":
            got = oracle.cd16(oracle.bf16_encode(x), q)
        else:
            got = oracle.cd8(x, c["scale"], q)
        assert float(got) == c["expected"], (c, float(got))


@pytest.mark.parametrize("d", [1, 3, 4, 8, 31, 32, 96, 100, 128, 768])
def test_distance_integer_data_exact(d):
    """Integer data 0..255 (the SIFT-shaped workload): every partial sum is
    an integer below 2^24, so the float32 result equals the exact one in any
    order; bfloat16 also holds 0..255 exactly."""
    rng = np.random.default_rng(d)
    X = rng.integers(0, 256, size=(200, d)).astype(np.float32)
    Qv = rng.integers(0, 256, size=(5, d)).astype(np.float32)
    for q in Qv:
        exact = ((X.astype(np.float64) - q) ** 2).sum(1)
        for i in range(len(X)):
            assert float(oracle.cd32(X[i], q)) == exact[i]
            assert float(oracle.cd16(oracle.bf16_encode(X[i]), q)) == exact[i]


def test_distance_fp8_exact_values():
    """Codes of small integers with scale 1 decode exactly; with integer
    queries the fp8 distance equals the exact one."""
    vals = oracle.e4m3_values()
    ints = [c for c in range(127) if float(vals[c]).is_integer() and vals[c] <= 16]
    rng = np.random.default_rng(7)
    for d in (16, 48, 768):
        codes = rng.choice(np.array(ints, np.uint8), size=d)
        q = rng.integers(0, 17, size=d).astype(np.float32)
        exact = float(((vals[codes].astype(np.float64) - q) ** 2).sum())
        assert float(oracle.cd8(codes, 1.0, q)) == exact


@pytest.mark.parametrize("d", [2, 5, 32, 96, 128, 768, 1000])
def test_distance_error_bound(d):
    """All terms are non-negative, so to first order the float32 result is
    within (2 + chunks-per-lane*W + log2 G) unit roundoffs of the float64
    value (difference, fma chain, pair tree)."""
    rng = np.random.default_rng(100 + d)
    W = 4
    C = -(-d // W)
    G = min(64, 1 << (C - 1).bit_length())
    bound = (2 + (-(-C // G)) * W + math.log2(G)) * 2.0 ** -24 * 1.01
    for _ in range(50):
        x = rng.standard_normal(d).astype(np.float32)
        q = rng.standard_normal(d).astype(np.float32)
        exact = float(((x.astype(np.float64) - q) ** 2).sum())
        got = float(oracle.cd32(x, q))
        assert abs(got - exact) <= bound * exact + 1e-30


# ---------------------------------------------------------------- codecs

def test_codec_golden_cases():
    g = json.load(open(os.path.join(GOLD, "codec_cases.json")))
    xs = np.array([a for a, _ in g["bf16"]], np.float32)
    assert oracle.bf16_encode(xs).tolist() == [b for _, b in g["bf16"]]
    vals = oracle.e4m3_values()
    for code, v in g["e4m3_value"]:
        assert float(vals[code]) == v
    ys = np.array([a for a, _ in g["e4m3_encode"]], np.float32)
    assert oracle.e4m3_encode(ys).tolist() == [c for _, c in g["e4m3_encode"]]


def test_bf16_matches_torch():
    """torch's float32 -> bfloat16 cast rounds to nearest even as well."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32) * 100,
                        (rng.integers(0, 2 ** 16, 5000).astype(np.float32) + 0.5) / 7.0])
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(oracle.bf16_encode(x), ref)


def test_e4m3_matches_torch():
    """torch.float8_e4m3fn is the same OCP format: equal values for every
    finite code, and equal nearest-even encodings inside [-448, 448]."""
    torch = pytest.importorskip("torch")
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float32).numpy()
    mine = oracle.e4m3_values()
    finite = ~np.isnan(ref)
    assert np.array_equal(np.isnan(mine), ~finite)
    assert np.array_equal(mine[finite], ref[finite])
    rng = np.random.default_rng(5)
    y = np.concatenate([rng.uniform(-448, 448, 20000), rng.standard_normal(20000) * 0.05,
                        (mine[finite][:-1] + mine[finite][1:]) / 2]).astype(np.float32)
    y = y[np.abs(y) <= 448]
    ref_codes = torch.from_numpy(y).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = oracle.e4m3_encode(y)
    # torch keeps the sign of a negative value that rounds to zero (0x80);
    # the encoder here writes +0 for every zero.
    ref_codes = np.where(ref_codes == 0x80, 0, ref_codes)
    assert np.array_equal(got, ref_codes)


# ---------------------------------------------------------------- beam search

def _pre_post_index():
    """The graph of the PRE/POST example (Section 2.2): v0 is the entry,
    v2 is out of range and bridges v0 to q's nearest neighbour v3; without
    v2, the search can only walk v0 -> v4 -> v5.  Positions (attribute
    ranks): v2=0, v0=1, v1=2, v3=3, v4=4, v5=5; query range [1,5]."""
    coords = {  # name: (position, xy)
        "v2": (0, (3.0, 0.0)), "v0": (1, (4.0, 4.0)), "v1": (2, (6.0, 6.0)),
        "v3": (3, (1.0, 0.0)), "v4": (4, (0.0, 4.5)), "v5": (5, (0.0, 3.5))}
    edges = {"v0": ["v2", "v4", "v1"], "v2": ["v0", "v3"], "v3": ["v2"], "v4": ["v0", "v5"],
             "v5": ["v4"], "v1": ["v0"]}
    pos = {k: v[0] for k, v in coords.items()}
    X = np.zeros((6, 2), np.float32)
    for k, (p, xy) in coords.items():
        X[p] = xy
    adj = np.full((1, 6, 4), 0xFFFFFFFF, np.uint32)
    for k, nb in edges.items():
        adj[0, pos[k], :len(nb)] = [pos[v] for v in nb]
    ep = np.array([0xFFFFFFFF, pos["v0"]], np.uint32)
    ix = oracle.OracleIndex(6, 2, 4, 1, 1, 2, np.arange(6), np.arange(6.0), X, adj, ep)
    return ix, pos


def test_pre_post_worked_example():
    """POST reaches v3 through v2 (v0 -> v2 -> v3); PRE -- the same graph
    with the out-of-range v2 and its edges removed -- ends at v5 after
    v0 -> v4 -> v5 (Section 2.2, example of Fig. 2)."""
    ix, pos = _pre_post_index()
    q = np.zeros(2, np.float32)
    part = dict(depth=0, heap=1, a=0, b=5, x=1, y=5)
    d, p, vis, hops, st = oracle.search_part(ix, part, q, m=1, cap_p=16)
    assert st == 0 and p.tolist() == [pos["v3"]] and d.tolist() == [1.0]
    # hand trace: expand v0 (finds v2,v4,v1), v2 (finds v3), v3; then v4 > v3 stops it
    assert vis.tolist() == [pos["v0"], pos["v2"], pos["v4"], pos["v1"], pos["v3"]]
    assert hops == 3
    # PRE: drop v2 from the graph
    adj = np.full_like(ix.adj, 0xFFFFFFFF)
    for u in range(6):
        if u == pos["v2"]:
            continue
        keep = [v for v in ix.adj[0, u] if v != 0xFFFFFFFF and v != pos["v2"]]
        adj[0, u, :len(keep)] = keep            # same order, v2 left out
    pre = oracle.OracleIndex(6, 2, 4, 1, 1, 2, np.arange(6), np.arange(6.0), ix.vec, adj, ix.ep)
    d, p, vis, hops, st = oracle.search_part(pre, part, q, m=1, cap_p=16)
    assert p.tolist() == [pos["v5"]] and d.tolist() == [12.25]
    assert vis.tolist() == [pos["v0"], pos["v4"], pos["v1"], pos["v5"]]


def test_learned_features_worked_example():
    """The 12 probe features on the PRE/POST example, traced by hand: from
    q = (0,0) the squared distances are v3 1, v2 9, v5 12.25, v4 20.25,
    v0 32, v1 72.  After one expansion of the entry v0 (m = cap = 4):
    P = {v2 9, v4 20.25, v1 72}, Q = {v4 20.25, v0 32, v1 72} (v2 is out of
    range), V = {v0, v2, v4, v1} of which 3 are in range, and the next
    candidate is v2 (9).  With k = 2, a query width of 5 and one part."""
    ix, pos = _pre_post_index()
    part = dict(depth=0, heap=1, a=0, b=5, x=1, y=5)
    d, p, vis, hops, st, f = oracle.search_part_learned(
        ix, part, np.zeros(2, np.float32), ef_max=4, switch_hop=1, ef2=0, k=2, w_query=5,
        n_parts=1)
    assert st == 0 and f is not None
    want = [np.log2(5), np.log2(6), 5 / 6,        # filter width, node size, ratio
            np.log2(5), 0.0,                       # query width, parts - 1
            3 / 4, min(3 / 2, 4),                  # P fill of its cap, Q fill over k
            3 / 4,                                 # in-range share of V
            20.25 / 32, 32 / 32, 9 / 32,           # best and k-th in Q, best in P (ratios)
            np.log2(1 + 4)]                        # log2(1 + |V|)
    assert np.allclose(f, want, rtol=0, atol=1e-12), (f, want)
    # the search itself is unchanged by a features-only switch
    d0, p0, _, h0, _ = oracle.search_part(ix, part, np.zeros(2, np.float32), m=4, cap_p=4)
    assert p.tolist() == p0.tolist() and hops == h0


def test_learned_features_live_part():
    """P's fill counts only its live part, and no switch is taken when the
    search stops right at the end of the probe.  Hand trace on a line,
    q = 0, m = cap = 2, k = 2, node [0,4], query range [1,3]; positions
    f=0 (x=10, out of range), e=1 (x=2, the entry), a=2 (x=3), g=3 (x=-4),
    h=4 (x=5, out of range); edges e -> a, f; a -> g, h; f, g, h -> e.
    Squared distances: e 4, a 9, g 16, h 25, f 100.
    After one expansion (of e): V = {e, a, f}, P = {a 9, f 100},
    Q = {e 4, a 9} (full, worst 9).  The next candidate a (9) is not
    farther than the worst, so the search goes on and the features are
    taken; f (100) is farther than the worst of a full Q and can never be
    expanded, so the live fill of P is 1/2.
    After two expansions (a's neighbours g 16 and h 25 both lose to the
    full Q): P = {g 16, h 25}, whose best is farther than the worst (9):
    the search stops, so no features are taken."""
    X = np.array([[10.0], [2.0], [3.0], [-4.0], [5.0]], np.float32)
    adj = np.full((1, 5, 2), 0xFFFFFFFF, np.uint32)
    adj[0, 1] = [2, 0]
    adj[0, 2] = [3, 4]
    adj[0, 0, 0] = adj[0, 3, 0] = adj[0, 4, 0] = 1
    ep = np.array([0xFFFFFFFF, 1], np.uint32)
    ix = oracle.OracleIndex(5, 1, 2, 1, 1, 2, np.arange(5), np.arange(5.0), X, adj, ep)
    part = dict(depth=0, heap=1, a=0, b=4, x=1, y=3)
    q = np.zeros(1, np.float32)
    d, p, vis, hops, st, f = oracle.search_part_learned(ix, part, q, ef_max=2, switch_hop=1,
                                                        ef2=0, k=2, w_query=3, n_parts=1)
    assert st == 0 and f is not None
    want = [np.log2(3), np.log2(5), 3 / 5, np.log2(3), 0.0,
            1 / 2,                                 # live part of P: a only
            1.0, 2 / 3,                            # Q fill over k, in-range share of V
            4 / 4, 9 / 4, 9 / 9,                   # best and k-th in Q, best in P
            np.log2(1 + 3)]
    assert np.allclose(f, want, rtol=0, atol=1e-12), (f, want)
    assert p.tolist() == [1, 2] and hops == 2 and vis.tolist() == [1, 2, 0, 3, 4]
    d, p, vis, hops, st, f = oracle.search_part_learned(ix, part, q, ef_max=2, switch_hop=2,
                                                        ef2=0, k=2, w_query=3, n_parts=1)
    assert st == 0 and f is None and hops == 2


def test_post_short_q_keeps_searching():
    """Alg. 1 stop test read with a full-Q guard: under POST, Q holds only
    in-range points, so it may be short of m while an out-of-range
    candidate is farther than everything in Q.  The search must go on
    through that candidate (otherwise in-range points behind it are lost).
    Hand trace on a 1-D line, q = 0, m = 2, range = positions [1,2]:
    entry e (x=1, in range) -> bridge b (x=5, out of range) -> t (x=-3, in
    range).  Q = {e} after the first hop; b (25) is farther than e (1) but
    Q is not full, so b is expanded and t (9) is found: answer [e, t]."""
    X = np.array([[5.0], [1.0], [-3.0]], np.float32)       # positions: b=0, e=1, t=2
    adj = np.full((1, 3, 2), 0xFFFFFFFF, np.uint32)
    adj[0, 1, 0] = 0          # e -> b
    adj[0, 0, :2] = [1, 2]    # b -> e, t
    adj[0, 2, 0] = 0          # t -> b
    ep = np.array([0xFFFFFFFF, 1], np.uint32)
    ix = oracle.OracleIndex(3, 1, 2, 1, 1, 2, np.arange(3), np.arange(3.0), X, adj, ep)
    part = dict(depth=0, heap=1, a=0, b=2, x=1, y=2)
    d, p, vis, hops, st = oracle.search_part(ix, part, np.zeros(1, np.float32), m=2, cap_p=4)
    assert p.tolist() == [1, 2] and d.tolist() == [1.0, 9.0]
    assert vis.tolist() == [1, 0, 2] and hops == 3


def _int_workload(n, d, seed, vmax=4):
    rng = np.random.default_rng(seed)
    return rng.integers(0, vmax, size=(n, d)).astype(np.float32), rng


@pytest.mark.parametrize("seed", range(4))
def test_exhaustive_search_equals_bruteforce(seed):
    """Finding 1 (Section 3.2): a graph built on a superset answers the
    range query; with m >= node size and a connected graph, Alg. 1 + POST
    visits the whole node and returns exactly the filtered k-NN.  Integer
    data (few values, many exact ties) makes float32 distances exact, so
    the answer equals the float64 brute force, ties broken by position."""
    X, rng = _int_workload(300, 6, seed)
    ix = make_test_index(X, leaf=8, R=6, ep_mode="random", rng=rng)
    for _ in range(40):
        l = int(rng.integers(0, 300))
        r = int(rng.integers(l, 300))
        q = rng.integers(0, 4, size=6).astype(np.float32)
        k = int(rng.integers(1, 12))
        parts, _ = oracle.select(300, 8, l, r)
        for p in parts:
            if p["kind"] != oracle.KIND_GRAPH:
                continue
            size = p["b"] - p["a"] + 1
            dd, pp, vis, hops, st = oracle.search_part(ix, p, q, m=size, cap_p=size)
            assert st == 0
            assert sorted(vis.tolist()) == list(range(p["a"], p["b"] + 1))
            gp, gd = oracle.bruteforce(ix.vec, q, p["x"], p["y"], size)
            w = p["y"] - p["x"] + 1
            assert pp.tolist() == gp[0][:w].tolist()
            assert np.array_equal(dd.astype(np.float64), gd[0][:w])
        ids, dists, stats, st = oracle.query(ix, q, l, r, k, ef=300, cap_p=300)
        gp, gd = oracle.bruteforce(ix.vec, q, l, r, k)
        assert ids.tolist() == gp[0].tolist()


@pytest.mark.parametrize("seed", range(3))
def test_search_invariants(seed):
    """Alg. 1 invariants at small ef: results lie in the part's range, are
    sorted by (distance, position) and unique; Q never exceeds m; every
    visited point is the entry or a neighbour of an earlier expanded point,
    so |V| <= 1 + hops * R; a hop budget of 0 returns only the entry."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((400, 8)).astype(np.float32)
    ix = make_test_index(X, leaf=16, R=6, ep_mode="random", rng=rng)
    for _ in range(60):
        l = int(rng.integers(0, 400))
        r = int(rng.integers(l, 400))
        q = rng.standard_normal(8).astype(np.float32)
        m = int(rng.integers(1, 20))
        for p in oracle.select(400, 16, l, r)[0]:
            if p["kind"] != oracle.KIND_GRAPH:
                continue
            dd, pp, vis, hops, st = oracle.search_part(ix, p, q, m=m, cap_p=m)
            assert st == 0 and len(pp) <= m
            assert np.all((pp >= p["x"]) & (pp <= p["y"]))
            keys = list(zip(dd.tolist(), pp.tolist()))
            assert keys == sorted(keys) and len(set(pp.tolist())) == len(pp)
            assert len(set(vis.tolist())) == len(vis) <= 1 + hops * ix.degree
            assert np.all((vis >= p["a"]) & (vis <= p["b"]))
            for j, pj in enumerate(pp):
                assert float(dd[j]) == float(oracle.cd32(ix.vec[pj], q))
            d0, p0, v0, h0, _ = oracle.search_part(ix, p, q, m=m, cap_p=m, hop_budget=0)
            e = int(ix.ep[p["heap"]])
            assert h0 == 0 and v0.tolist() == [e]
            assert p0.tolist() == ([e] if p["x"] <= e <= p["y"] else [])


def test_query_merges_parts():
    """Alg. 4's last step: the answer is the top k, by (distance, position),
    of the parts' answers."""
    rng = np.random.default_rng(11)
    X = rng.standard_normal((500, 8)).astype(np.float32)
    ix = make_test_index(X, leaf=10, R=6)
    seen2 = 0
    for _ in range(80):
        l = int(rng.integers(0, 500))
        r = int(rng.integers(l, 500))
        q = rng.standard_normal(8).astype(np.float32)
        k, ef = 5, 12
        parts, cnt = oracle.select(500, 10, l, r)
        pool = []
        for p in parts:
            if p["kind"] == oracle.KIND_GRAPH:
                dd, pp, _, _, _ = oracle.search_part(ix, p, q, m=ef, cap_p=ef)
            else:
                pp = np.arange(p["x"], p["y"] + 1)
                dd = np.array([oracle.cd32(ix.vec[i], q) for i in pp], np.float32)
            pool += list(zip(dd.tolist(), pp.tolist()))
        seen2 += cnt == 2
        ids, dists, stats, st = oracle.query(ix, q, l, r, k, ef)
        best = sorted(pool)[:k]
        got = [(float(a), int(b)) for a, b in zip(dists, ids) if b >= 0]
        assert got == best
        assert stats[0] == cnt
    assert seen2 > 0


@pytest.mark.parametrize("seed", range(2))
def test_learned_switch_special_cases(seed):
    """The learned switch reduces to plain Alg. 1 in three special cases:
    a new beam equal to the old one changes nothing; a switch at hop 0 to
    beam e is the search with ef = e from the start; granting G further
    expansions after s hops is the per-part hop budget s + G."""
    rng = np.random.default_rng(20 + seed)
    X = rng.standard_normal((600, 8)).astype(np.float32)
    ix = make_test_index(X, leaf=12, R=6, ep_mode="random", rng=rng)
    cut = 0
    for _ in range(50):
        l = int(rng.integers(0, 600))
        r = int(rng.integers(l, 600))
        q = rng.standard_normal(8).astype(np.float32)
        k, ef, s = 5, 24, int(rng.integers(1, 6))
        base = oracle.query(ix, q, l, r, k, ef)
        same = oracle.query_learned(ix, q, l, r, k, ef, s, np.array([ef, ef], np.int32))
        assert same[0].tolist() == base[0].tolist() and same[1].tolist() == base[1].tolist()
        assert same[2][1] == base[2][1]
        e = int(rng.integers(k, ef))
        small = oracle.query(ix, q, l, r, k, e)
        sw0 = oracle.query_learned(ix, q, l, r, k, ef, 0, np.array([e, e], np.int32))
        assert sw0[0].tolist() == small[0].tolist() and sw0[2][1] == small[2][1]
        g = int(rng.integers(1, 8))
        budget = oracle.query(ix, q, l, r, k, ef, hop_budget=s + g)
        stop = oracle.query_learned(ix, q, l, r, k, ef, s, np.zeros(2, np.int32),
                                    hop2_parts=np.array([g, g]))
        assert stop[0].tolist() == budget[0].tolist() and stop[2][1] == budget[2][1]
        cut += budget[2][1] < base[2][1]
    assert cut > 10


# ---------------------------------------------------------------- brute force

def test_bruteforce_matches_sort_definition():
    """Def. 2.2 written with library primitives: all distances in float64,
    positions filtered to [l,r], lexicographic sort by (distance, position)."""
    rng = np.random.default_rng(21)
    X = rng.integers(0, 3, size=(800, 5)).astype(np.float32)   # many ties
    for _ in range(50):
        l = int(rng.integers(0, 800))
        r = int(rng.integers(l, 800))
        q = rng.integers(0, 3, size=5).astype(np.float32)
        k = int(rng.integers(1, 30))
        D = ((X.astype(np.float64) - q) ** 2).sum(1)
        pos = np.arange(800)
        sel = (pos >= l) & (pos <= r)
        order = np.lexsort((pos[sel], D[sel]))
        want = pos[sel][order][:k]
        gp, gd = oracle.bruteforce(X, q, l, r, k)
        assert gp[0][:len(want)].tolist() == want.tolist()
        assert np.all(gp[0][len(want):] == -1)


def test_lemma_3_1_containment():
    """Lemma 3.1: if the unfiltered h nearest neighbours hold at least k
    in-range points, the range-filtered k-NN set lies inside them."""
    rng = np.random.default_rng(31)
    X = rng.standard_normal((2000, 6)).astype(np.float32)
    checked = 0
    for _ in range(100):
        l = int(rng.integers(0, 1500))
        r = int(rng.integers(l, 2000))
        q = rng.standard_normal(6).astype(np.float32)
        k = 10
        h = int(rng.integers(10, 400))
        hp, _ = oracle.bruteforce(X, q, 0, 1999, h)
        inr = hp[0][(hp[0] >= l) & (hp[0] <= r)]
        if len(inr) >= k:
            kp, _ = oracle.bruteforce(X, q, l, r, k)
            assert set(kp[0].tolist()) <= set(hp[0].tolist())
            checked += 1
    assert checked > 10


def test_expected_examined_points():
    """Section 4.2 (fanout extension): with attributes independent of the
    vectors, the number of points examined in distance order until k
    in-range ones appear has mean k(L+1)/(w+1) (L node size, w in-range
    count; the negative hypergeometric mean)."""
    rng = np.random.default_rng(41)
    L, w, k = 1024, 256, 10
    X = rng.standard_normal((L, 4)).astype(np.float32)
    ranks = []
    for _ in range(400):
        q = rng.standard_normal(4).astype(np.float32)
        perm = rng.permutation(L)          # attribute ranks independent of vectors
        Xp = X[perm]
        allp, _ = oracle.bruteforce(Xp, q, 0, L - 1, L)
        inr = np.flatnonzero((allp[0] >= 100) & (allp[0] < 100 + w))
        ranks.append(inr[k - 1] + 1)
    mean = float(np.mean(ranks))
    expect = k * (L + 1) / (w + 1)
    sd = float(np.std(ranks)) / math.sqrt(len(ranks))
    assert abs(mean - expect) < 4 * sd


def test_recall_definition():
    rng = np.random.default_rng(51)
    X = rng.standard_normal((300, 4)).astype(np.float32)
    Q = rng.standard_normal((5, 4)).astype(np.float32)
    l = np.array([0, 10, 20, 290, 0])
    r = np.array([299, 200, 25, 299, 0])
    gp, gd = oracle.bruteforce(X, Q, l, r, 10)
    rec, strict, per = oracle.recall(X, Q, l, r, gp, gp, gd, 10)
    assert rec == 1.0 and strict == 1.0
    bad = gp.copy()
    bad[0, 0] = -1
    rec2, _, per2 = oracle.recall(X, Q, l, r, bad, gp, gd, 10)
    assert per2[0] == 0.9 and per2[4] == 1.0   # a 1-point range needs only 1 hit


# ---------------------------------------------------------------- beam-width network

def test_mlp_backprop_matches_finite_differences():
    """The float64 manual backward of the 12-64-64-1 ReLU network equals
    central finite differences of its forward (loss = mean squared error)."""
    rng = np.random.default_rng(61)
    params = np.concatenate([rng.standard_normal(5057) * 0.2, rng.standard_normal(12),
                             np.abs(rng.standard_normal(12)) + 0.5])
    F = rng.standard_normal((40, 12)) * 2.0
    T = rng.standard_normal(40)
    grad, loss = oracle.mlp_grad64(params, F, T)

    def L(p):
        y, _ = oracle.mlp_forward64(p, F)
        return np.mean((y - T) ** 2)

    assert abs(L(params) - loss) < 1e-12
    idx = np.concatenate([rng.choice(768, 30), 768 + rng.choice(64, 8), 832 + rng.choice(4096, 30),
                          4928 + rng.choice(64, 8), 4992 + rng.choice(64, 10), [5056]])
    h = 1e-6
    for j in idx:
        e = np.zeros_like(params)
        e[j] = h
        fd = (L(params + e) - L(params - e)) / (2 * h)
        assert abs(fd - grad[j]) <= 1e-6 + 1e-5 * abs(fd), (j, fd, grad[j])


# ---------------------------------------------------------------- Adam

def test_adam_first_step_is_sign_step():
    """Step 1 from zero moments: both bias corrections cancel the (1 - beta)
    factors exactly, so the update is lr * g / (|g| + eps): lr times the
    sign of g wherever |g| >> eps.  A wrong or missing bias correction
    scales it by (1 - beta1) / sqrt(1 - beta2) or its inverse."""
    rng = np.random.default_rng(11)
    g = rng.standard_normal(500) * np.exp(rng.uniform(-8, 4, 500))
    theta = rng.standard_normal(500)
    lr = 1e-3
    t1, m, v = oracle.adam_step64(theta, g, np.zeros(500), np.zeros(500), 1, lr)
    assert np.allclose(theta - t1, lr * g / (np.abs(g) + oracle.ADAM_EPS), rtol=1e-12, atol=0)
    assert np.allclose(m, (1 - oracle.ADAM_B1) * g, rtol=1e-15)
    assert np.allclose(v, (1 - oracle.ADAM_B2) * g * g, rtol=1e-15)


def test_adam_constant_gradient_keeps_its_step():
    """With the same gradient at every step from zero moments, the biased
    moments are (1 - beta^t) g and (1 - beta^t) g^2, so the bias-corrected
    ones are exactly g and g^2 and every step moves by lr * g / (|g| + eps)
    (Kingma and Ba, Section 3: the correction removes the initialisation
    bias).  A wrong decay rate or exponent in the correction drifts."""
    rng = np.random.default_rng(12)
    g = rng.standard_normal(300)
    theta = rng.standard_normal(300)
    m = np.zeros(300)
    v = np.zeros(300)
    lr = 2e-3
    step = lr * g / (np.abs(g) + oracle.ADAM_EPS)
    for t in range(1, 60):
        t1, m, v = oracle.adam_step64(theta, g, m, v, t, lr)
        assert np.allclose(theta - t1, step, rtol=1e-9, atol=0), t
        theta = t1
    assert np.allclose(m, (1 - oracle.ADAM_B1 ** 59) * g, rtol=1e-12)


def test_adam_zero_gradient_after_one_step():
    """After a step with g, a zero gradient at step 2 leaves
    m = beta1 (1 - beta1) g and v = beta2 (1 - beta2) g^2, so the second
    update is lr * [beta1 (1-beta1) g / (1-beta1^2)] /
    (sqrt(beta2 (1-beta2) g^2 / (1-beta2^2)) + eps), worked from the
    definitions: the momentum keeps moving the point."""
    b1, b2, eps = oracle.ADAM_B1, oracle.ADAM_B2, oracle.ADAM_EPS
    g = np.array([0.5, -2.0, 1e-3])
    theta = np.zeros(3)
    t1, m, v = oracle.adam_step64(theta, g, np.zeros(3), np.zeros(3), 1, 0.01)
    t2, m, v = oracle.adam_step64(t1, np.zeros(3), m, v, 2, 0.01)
    mh = b1 * (1 - b1) * g / (1 - b1 ** 2)
    vh = b2 * (1 - b2) * g * g / (1 - b2 ** 2)
    assert np.allclose(t1 - t2, 0.01 * mh / (np.sqrt(vh) + eps), rtol=1e-12)
