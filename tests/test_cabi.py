"""Host-side checks of libesg (no GPU needed): exported symbols, status
strings, the index builder's output structure and determinism, and the
loader's rejection of malformed files."""
from __future__ import annotations

import ctypes
import os
import re
import shutil
import struct

import numpy as np
import pytest

import oracle
import synth
import paper_2504_04018_amd as esg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported():
    txt = open(os.path.join(ROOT, "include", "esg.h")).read()
    names = set(re.findall(r"^\s*(?:int32_t|void|const char\*)\s+(esg_\w+)\s*\(", txt, re.M))
    assert len(names) >= 9
    L = esg.lib()
    for n in names:
        assert hasattr(L, n), n
    assert names <= set(esg.SIGNATURES), names - set(esg.SIGNATURES)


def test_status_strings():
    for s in range(0, -9, -1):
        assert esg.status_str(s).startswith("ESG")
    assert "unknown" in esg.status_str(-99)


@pytest.fixture(scope="module")
def small_index(tmp_path_factory):
    w = synth.make_workload(0, n=3000, nq=0)
    d = tmp_path_factory.mktemp("cabi")
    path = str(d / "s.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=12, leaf=100,
                    ef_construction=64)
    return w, path


@pytest.fixture(scope="module", params=[2, 4, 16])
def fanout_index(request, tmp_path_factory):
    f = request.param
    w = synth.make_workload(0, n=3000, nq=0)
    path = str(tmp_path_factory.mktemp(f"cabi_f{f}") / "s.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=12, leaf=100,
                    ef_construction=64, fanout=f)
    return w, path, f


def test_builder_structure(fanout_index):
    """Alg. 3 output on a fanout-f tree (f = 2, 4, 16; Section 4.2,
    Extensions): one graph per tree node with b-a >= leaf, neighbours inside
    the node, no self loops or repeats, degree <= R, rows packed, entry point
    inside the node, position order = attribute order, c = 1/f."""
    w, path, f = fanout_index
    ix = oracle.read_index(path)
    assert ix.fanout == f and ix.c_den == f
    assert np.array_equal(np.sort(w["attr"]), ix.attr)
    assert np.array_equal(ix.vec, w["X"][ix.ext_id])
    from tests.helpers import tree_nodes
    depth_seen = set()
    for t, h, a, b, g in tree_nodes(ix.n, ix.leaf, f):
        if not g:
            continue
        depth_seen.add(t)
        e = int(ix.ep[h])
        assert a <= e <= b
        rows = ix.adj[t, a:b + 1]
        valid = rows != oracle.NO_NODE
        # packed: no valid entry after a pad
        assert np.all(np.diff(valid.astype(int), axis=1) <= 0)
        vals = rows[valid].astype(np.int64)
        assert np.all((vals >= a) & (vals <= b))
        for i, row in enumerate(rows):
            rv = row[row != oracle.NO_NODE]
            assert len(set(rv.tolist())) == len(rv) and (a + i) not in rv.tolist()
        assert valid.sum(1).min() >= 1
    assert depth_seen == set(range(ix.n_depth))
    # rows of positions outside every graph node of a depth stay empty
    for t in range(ix.n_depth):
        covered = np.zeros(ix.n, bool)
        for tt, h, a, b, g in tree_nodes(ix.n, ix.leaf, f):
            if tt == t and g:
                covered[a:b + 1] = True
        assert np.all(ix.adj[t][~covered] == oracle.NO_NODE)
    # the tree is shallower at a larger fanout: 3000 points, leaf 100
    assert ix.n_depth == {2: 5, 4: 3, 16: 2}[f]


def test_fanout_index_oracle_invariants(fanout_index):
    """The oracle's search on a fanout-f index: at most two parts per query
    (Lemma 4.3), every answer inside [l,r], and an exhaustive beam
    (ef >= every node size) equals the float64 brute force (Finding 1)."""
    w, path, f = fanout_index
    ix = oracle.read_index(path)
    rng = np.random.default_rng(f)
    Q = synth.make_workload(0, n=3000, nq=40)["Q"]
    wd = np.rint(np.exp(rng.uniform(0, np.log(3000), 40))).astype(np.int64)
    l = (rng.random(40) * (3000 - wd + 1)).astype(np.int64)
    r = l + wd - 1
    ids, dists, st, stats = oracle.query_batch(ix, Q, l, r, 10, 4096, 4096, with_stats=True)
    assert np.all(st == 0) and np.all(stats[:, 0] <= 2)
    pos_of = np.empty(ix.n, np.int64)
    pos_of[ix.ext_id] = np.arange(ix.n)
    pos = np.where(ids >= 0, pos_of[np.maximum(ids, 0)], -1)
    assert np.all((pos == -1) | ((pos >= l[:, None]) & (pos <= r[:, None])))
    gt_pos, gt_d = oracle.bruteforce(ix.vec, Q, l, r, 10)
    rec, _, _ = oracle.recall(ix.vec, Q, l, r, pos, gt_pos, gt_d, 10)
    assert rec == 1.0


@pytest.fixture(scope="module", params=[2, 3])
def chain_index(request, tmp_path_factory):
    B = request.param
    w = synth.make_workload(0, n=3000, nq=0)
    path = str(tmp_path_factory.mktemp(f"chain{B}") / "c.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=12, leaf=100,
                    ef_construction=64, fanout=B, layout="chain")
    return w, path, B


def test_chain_builder_structure(chain_index, tmp_path):
    """The half-bounded index (Section 4.1, Alg. 2): one graph per recorded
    prefix [0, s_i - 1] and suffix [n - s_i, n - 1] (s_0 = n,
    s_{i+1} = ceil(s_i / B), while s_i - 1 >= leaf); neighbours and entry
    inside the recorded range, no self loops or repeats; O(N) rows in all
    (2 sum s_i < 4N per chain pair); independent of the thread count."""
    w, path, B = chain_index
    ix = oracle.read_index(path)
    assert ix.layout == 1 and ix.fanout == B and ix.c_den == B
    sizes, starts = oracle.chain_levels(ix.n, ix.leaf, B)
    assert ix.n_depth == len(sizes) and sizes[0] == ix.n
    assert ix.adj.size == sum(sizes) * ix.degree and sum(sizes) < 2 * ix.n * B / (B - 1) + 4 * len(sizes)
    for t, (sz, a) in enumerate(zip(sizes, starts)):
        b = a + sz - 1
        e = int(ix.ep[t + 1])
        assert a <= e <= b
        rows = ix.rows(t)[a:b + 1]
        valid = rows != oracle.NO_NODE
        assert np.all(np.diff(valid.astype(int), axis=1) <= 0)
        vals = rows[valid].astype(np.int64)
        assert np.all((vals >= a) & (vals <= b))
        for i, row in enumerate(rows):
            rv = row[row != oracle.NO_NODE].tolist()
            assert len(set(rv)) == len(rv) and (a + i) not in rv
    p1 = str(tmp_path / "c1.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), p1, degree=12, leaf=100,
                    ef_construction=64, fanout=B, layout="chain", threads=1)
    assert open(p1, "rb").read() == open(path, "rb").read()
    assert _load_status(path) in (esg.ESG_OK, esg.ESG_EHIP)


def test_chain_index_exhaustive_equals_bruteforce(chain_index):
    """Finding 1 on the half-bounded index: with a beam as large as the
    recorded range, the search of the chosen prefix or suffix graph under
    POST returns the exact filtered k-NN, for prefix, suffix and general
    ranges; every query takes one part."""
    w, path, B = chain_index
    ix = oracle.read_index(path)
    n = ix.n
    Q = synth.make_workload(0, n=3000, nq=60)["Q"]
    rng = np.random.default_rng(B)
    r = rng.integers(0, n, 60)
    l = np.where(np.arange(60) % 3 == 0, 0, np.where(np.arange(60) % 3 == 1, r, rng.integers(0, n, 60)))
    l, r = np.minimum(l, r), np.where(np.arange(60) % 3 == 1, n - 1, np.maximum(l, r))
    ids, dists, st, stats = oracle.query_batch(ix, Q, l, r, 10, 4096, 4096, with_stats=True)
    assert np.all(st == 0) and np.all(stats[:, 0] == 1)
    pos_of = np.empty(n, np.int64)
    pos_of[ix.ext_id] = np.arange(n)
    pos = np.where(ids >= 0, pos_of[np.maximum(ids, 0)], -1)
    gt_pos, gt_d = oracle.bruteforce(ix.vec, Q, l, r, 10)
    rec, _, _ = oracle.recall(ix.vec, Q, l, r, pos, gt_pos, gt_d, 10)
    assert rec == 1.0


def test_builder_fanout_errors(tmp_path):
    X = np.zeros((10, 4), np.float32)
    with pytest.raises(esg.EsgError) as e:
        esg.build_index(X, np.arange(10.0), str(tmp_path / "x"), fanout=1)
    assert e.value.status == esg.ESG_EINVAL
    with pytest.raises(esg.EsgError) as e:
        esg.build_index(X, np.arange(10.0), str(tmp_path / "x"), fanout=65)
    assert e.value.status == esg.ESG_EUNSUPPORTED


def test_builder_deterministic(small_index, tmp_path):
    w, path = small_index
    p1 = str(tmp_path / "t1.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), p1, degree=12, leaf=100,
                    ef_construction=64, threads=1)
    assert open(p1, "rb").read() == open(path, "rb").read()


def test_builder_errors(tmp_path):
    X = np.zeros((10, 4), np.float32)
    with pytest.raises(esg.EsgError) as e:
        esg.build_index(X, np.arange(10.0), str(tmp_path / "x"), leaf=0)
    assert e.value.status == esg.ESG_EINVAL
    with pytest.raises(esg.EsgError) as e:
        esg.build_index(X, np.full(10, np.nan), str(tmp_path / "x"))
    assert e.value.status == esg.ESG_EINVAL
    with pytest.raises(esg.EsgError) as e:
        esg.build_index(X, np.arange(10.0), "/nonexistent_dir/x.esgi")
    assert e.value.status == esg.ESG_EIO


def _crc32c(data: bytes) -> int:
    """CRC-32C (Castagnoli, reflected polynomial 0x82F63B78), bit by bit."""
    crc = 0xFFFFFFFF
    for byte in data:
        crc ^= byte
        for _ in range(8):
            crc = (crc >> 1) ^ (0x82F63B78 if crc & 1 else 0)
    return crc ^ 0xFFFFFFFF


def test_crc32c_check_value():
    # the standard check value of CRC-32C over the ASCII digits 1..9
    assert _crc32c(b"123456789") == 0xE3069283


def _load_status(path):
    import ctypes
    h = ctypes.c_void_p()
    st = esg.lib().esg_load_index(path.encode(), 0, ctypes.byref(h))
    if st == 0:
        esg.lib().esg_free_index(h)
    return st


def test_loader_rejects_malformed(small_index, tmp_path):
    w, path = small_index
    raw = bytearray(open(path, "rb").read())
    assert _load_status(str(tmp_path / "missing.esgi")) == esg.ESG_EIO

    def variant(name, data):
        p = str(tmp_path / name)
        open(p, "wb").write(bytes(data))
        return _load_status(p)

    bad = raw.copy(); bad[0] ^= 1
    assert variant("magic", bad) == esg.ESG_EFORMAT
    assert variant("trunc", raw[:-100]) == esg.ESG_EFORMAT
    bad = raw.copy(); bad[-8] ^= 0x40                      # entry-point section byte
    assert variant("crc", bad) == esg.ESG_EFORMAT
    bad = raw.copy(); bad[20] ^= 1                          # header field (n)
    assert variant("hdr", bad) == esg.ESG_EFORMAT
    # c = 1 / c_den above 1 / fanout: Alg. 4 could select more than two parts
    # (Lemma 4.2 needs c <= 1/2); a consistent header (checksum rewritten)
    # with c_den = 1 must still be refused
    bad = raw.copy()
    assert struct.unpack_from("<i", bad, 44)[0] == 2        # c_den
    struct.pack_into("<i", bad, 44, 1)
    struct.pack_into("<I", bad, 140, _crc32c(bytes(bad[:140])))
    assert variant("cden", bad) == esg.ESG_EFORMAT
    # metric fields (offset 124: metric, dq; 132: M^2) that disagree with
    # each other or with d, each behind a valid checksum
    assert struct.unpack_from("<2i", raw, 124) == (0, struct.unpack_from("<i", raw, 24)[0])
    d = struct.unpack_from("<i", raw, 24)[0]
    for name, metric, dq, m2 in [("metric", 3, d, 0.0), ("ip_dq", 2, d, 1.0),
                                 ("l2_m2", 0, d, 1.0), ("ang_dq", 1, d - 1, 0.0),
                                 ("ip_nan", 2, d - 1, float("nan"))]:
        bad = raw.copy()
        struct.pack_into("<2id", bad, 124, metric, dq, m2)
        struct.pack_into("<I", bad, 140, _crc32c(bytes(bad[:140])))
        assert variant(name, bad) == esg.ESG_EFORMAT, name
    # a well-formed file: loads where a device exists, reports the missing device here
    assert _load_status(path) in (esg.ESG_OK, esg.ESG_EHIP)


@pytest.fixture(scope="module", params=["ip", "angular"])
def metric_index(request, tmp_path_factory):
    m = request.param
    w = synth.make_workload(0, n=3000, nq=80)
    X = synth.spread_norms(w["X"], 0.5, 11)
    path = str(tmp_path_factory.mktemp(f"cabi_{m}") / "s.esgi")
    esg.build_index(X, w["attr"].astype(np.float64), path, degree=12, leaf=100,
                    ef_construction=64, metric=m)
    return w, X, path, {"ip": oracle.METRIC_IP, "angular": oracle.METRIC_ANGULAR}[m]


def test_metric_builder_stores_transform(metric_index):
    """The stored rows are the float64 transform rounded to float32 (unit
    rows; [x, sqrt(M^2 - |x|^2)]), in position order; the header carries the
    metric, the query length and M^2."""
    w, X, path, metric = metric_index
    ix = oracle.read_index(path)
    S, m2 = oracle.metric_store64(X, metric)
    assert ix.metric == metric and ix.d == S.shape[1]
    assert ix.dq == X.shape[1]
    assert ix.max_norm2 == pytest.approx(m2, rel=1e-13, abs=0)
    want = S[ix.ext_id].astype(np.float32)
    assert np.allclose(ix.vec, want, rtol=2e-7, atol=1e-6 * np.sqrt(max(m2, 1.0)))


def test_metric_index_oracle_recall(metric_index):
    """End to end on the CPU: the oracle's Alg. 4 + Alg. 1 search over the
    stored rows with dq-long queries finds the exact top 10 of the metric
    (largest inner product, or cosine) over the original rows."""
    w, X, path, metric = metric_index
    ix = oracle.read_index(path)
    Q, l, r = w["Q"], w["l"], w["r"]
    ids, _, st = oracle.query_batch(ix, Q, l, r, 10, 128)
    assert np.all(st == 0)
    pos_of = np.empty(ix.n, np.int64)
    pos_of[ix.ext_id] = np.arange(ix.n)
    Xpos = X[ix.ext_id]
    gt, _ = oracle.exact_metric(Xpos, Q, l, r, 10, metric)
    hit = 0
    tot = 0
    for i in range(len(Q)):
        g = gt[i][gt[i] >= 0]
        f = pos_of[ids[i][ids[i] >= 0]]
        hit += len(np.intersect1d(g, f))
        tot += len(g)
    assert hit / tot >= 0.95


def test_metric_builder_errors(tmp_path):
    X = np.ones((10, 4), np.float32)
    X[3] = 0
    with pytest.raises(esg.EsgError) as e:      # a zero row has no direction
        esg.build_index(X, np.arange(10.0), str(tmp_path / "x"), metric="angular")
    assert e.value.status == esg.ESG_EINVAL
    X[3] = np.inf
    with pytest.raises(esg.EsgError) as e:
        esg.build_index(X, np.arange(10.0), str(tmp_path / "x"), metric="ip")
    assert e.value.status == esg.ESG_EINVAL
    p = esg.BuildParams(16, 4, 16, 2, 1, 0, 0, 0, 7)
    st = esg.lib().esg_build_index(X.ctypes.data, np.arange(10.0).ctypes.data, 10, 4,
                                   ctypes.byref(p), str(tmp_path / "y").encode())
    assert st == esg.ESG_EINVAL


def test_gpu_builder_argument_checks(tmp_path):
    """The device builder's host-side checks, which run before any device
    call: a negative device and a node batch above 8,192 are refused; here
    (no HIP device) a valid call reports the missing device."""
    X = np.ones((50, 32), np.float32)
    p = esg.BuildParams(16, 8, 16, 2, 1, 0, 0, 0, 0)
    out = str(tmp_path / "g").encode()
    L = esg.lib()
    assert L.esg_build_index_gpu(X.ctypes.data, np.arange(50.0).ctypes.data, 50, 32,
                                 ctypes.byref(p), -1, out) == esg.ESG_EINVAL
    p.batch_max = 8193
    assert L.esg_build_index_gpu(X.ctypes.data, np.arange(50.0).ctypes.data, 50, 32,
                                 ctypes.byref(p), 0, out) == esg.ESG_EINVAL
    p.batch_max = 0
    st = L.esg_build_index_gpu(X.ctypes.data, np.arange(50.0).ctypes.data, 50, 32,
                               ctypes.byref(p), 0, out)
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except ImportError:
        has_gpu = False
    assert st == (esg.ESG_OK if has_gpu else esg.ESG_EHIP)
