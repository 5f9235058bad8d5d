"""GPU parity: the HIP search path against the CPU oracle, element by element.

Bar: integer results (parts, visited sets, hop counts, ids) bit-exact;
float32 distances bit-identical to the oracle's float32 distances (same
fixed summation order) and within 1e-5 relative of float64.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2504_04018_amd as esg  # noqa: E402

DEV = torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def tiny(tmp_path_factory):
    """Tiny workload (N=10,000, d=32, 200 queries), leaf bound 128."""
    w = synth.make_workload(0)
    path = str(tmp_path_factory.mktemp("tiny") / "tiny.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=16, leaf=w["leaf"],
                    ef_construction=200)
    gix = esg.Index(path, 0)
    oix = oracle.read_index(path)
    yield w, gix, oix, path
    gix.free()


@pytest.fixture(scope="module")
def tiny32(tmp_path_factory):
    """Tiny workload with degree 32 (rows of 32: full-width batches)."""
    w = synth.make_workload(0, n=6000, nq=120)
    path = str(tmp_path_factory.mktemp("tiny32") / "tiny32.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=32, leaf=100,
                    ef_construction=100)
    gix = esg.Index(path, 0)
    oix = oracle.read_index(path)
    yield w, gix, oix, path
    gix.free()


@pytest.fixture(scope="module")
def emb(tmp_path_factory):
    """Embedding-shaped workload at reduced size (N=12,000 unit-norm vectors
    in d=768, 40 queries, k=100 in the tests), degree 32, leaf bound 256."""
    w = synth.make_workload(3, n=12000, nq=40)
    path = str(tmp_path_factory.mktemp("emb") / "emb.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=32, leaf=256,
                    ef_construction=100)
    gix = esg.Index(path, 0)
    oix = oracle.read_index(path)
    yield w, gix, oix, path
    gix.free()


def gpu_search(gix, Q, l, r, k, ef, visited_cap=0, **kw):
    nq = len(Q)
    tr = esg.trace_tensor(nq, DEV)
    vis = None
    if visited_cap:
        vis = torch.zeros((nq * 2 * visited_cap,), dtype=torch.int32, device=DEV)
    ninv = torch.zeros(1, dtype=torch.int64, device=DEV)
    print(f"[gpu] search nq={nq} k={k} ef={ef} opts={kw}", flush=True)
    ids, dists = gix.search_ex(_t(Q), _t(l), _t(r), k, ef, trace=tr, visited=vis,
                               visited_cap=visited_cap, n_invalid=ninv, **kw)
    torch.cuda.synchronize()
    out = dict(ids=ids.cpu().numpy(), dists=dists.cpu().numpy(), trace=esg.decode_trace(tr),
               n_invalid=int(ninv.item()))
    if visited_cap:
        out["visited"] = vis.cpu().numpy().view(np.uint32).reshape(nq, 2, visited_cap)
    return out


def oracle_parts(oix, q, l, r, ef, cap_p, hop_budget=-1, kind=oracle.DIST_F32):
    parts, cnt = oix.select(l, r)
    res = []
    for p in parts:
        if p["kind"] == oracle.KIND_GRAPH:
            d, pp, vis, hops, st = oracle.search_part(oix, p, q, ef, cap_p, hop_budget, kind)
            assert st == 0
            res.append((p, set(vis.tolist()), hops, len(vis)))
        else:
            res.append((p, None, 0, p["y"] - p["x"] + 1))
    return res


def check_against_oracle(w, oix, out, Q, l, r, k, ef, cap_p=None, hop_budget=-1,
                         kind=oracle.DIST_F32, rerank=0, check_visited=True):
    cap = ef if not cap_p else cap_p
    oid, od, st = oracle.query_batch(oix, Q, l, r, k, ef, cap, hop_budget, kind, rerank)
    assert np.all(st == 0)
    bad = np.flatnonzero(np.any(out["ids"] != oid, axis=1))
    assert len(bad) == 0, f"ids differ for queries {bad[:10]}"
    assert np.array_equal(out["dists"].view(np.uint32), od.view(np.uint32)), "distances differ"
    tr = out["trace"]
    for i in range(len(Q)):
        parts = oracle_parts(oix, Q[i], int(l[i]), int(r[i]), ef, cap, hop_budget, kind)
        assert int(np.sum(tr["kind"][i] > 0)) == len(parts)
        for j, (p, vis, hops, nv) in enumerate(parts):
            got = {f: int(tr[f][i, j]) for f in ("kind", "depth", "heap", "a", "b", "x", "y")}
            assert got == p, (i, j, got, p)
            assert int(tr["hops"][i, j]) == hops, (i, j)
            assert int(tr["n_visited"][i, j]) == nv, (i, j)
            if check_visited and vis is not None and "visited" in out:
                cap_v = out["visited"].shape[2]
                if nv <= cap_v:
                    assert set(out["visited"][i, j, :nv].tolist()) == vis, (i, j)


def test_tiny_parity_full(tiny):
    """Tiny workload at its own k=10, ef=64: parts, visited sets, hops, ids
    and distances identical to the oracle; distances within 1e-5 of float64."""
    w, gix, oix, _ = tiny
    Q, l, r = w["Q"], w["l"], w["r"]
    out = gpu_search(gix, Q, l, r, w["k"], w["ef"], visited_cap=4096)
    check_against_oracle(w, oix, out, Q, l, r, w["k"], w["ef"])
    pos_of = np.empty(oix.n, np.int64)
    pos_of[oix.ext_id] = np.arange(oix.n)
    ids = out["ids"]
    ok = ids >= 0
    pos = np.where(ok, pos_of[np.maximum(ids, 0)], -1)
    assert np.all((pos[ok] >= np.repeat(l[:, None], w["k"], 1)[ok]) &
                  (pos[ok] <= np.repeat(r[:, None], w["k"], 1)[ok]))
    for i in range(len(Q)):
        d64 = oracle.exact_dist64(oix.vec, Q[i], pos[i][ok[i]])
        rel = np.abs(out["dists"][i][ok[i]].astype(np.float64) - d64) / np.maximum(d64, 1e-30)
        assert np.all(rel <= 1e-5)


@pytest.mark.parametrize("k,ef", [(1, 1), (10, 16), (5, 63), (10, 65), (32, 128), (100, 200),
                                  (10, 256), (64, 512), (100, 1024)])
def test_tiny_parity_k_ef(tiny, k, ef):
    """Every list width (ef up to 64, 128, 256, 512, 1024 words) and k."""
    w, gix, oix, _ = tiny
    n = 60
    Q, l, r = w["Q"][:n], w["l"][:n], w["r"][:n]
    out = gpu_search(gix, Q, l, r, k, ef, visited_cap=8192)
    check_against_oracle(w, oix, out, Q, l, r, k, ef)


@pytest.mark.parametrize("cap_p,hop_budget,hash_cap", [(1, -1, 0), (128, -1, 0), (64, 0, 0),
                                                       (64, 7, 0), (64, -1, 64), (32, 50, 128),
                                                       (64, -1, 256), (200, -1, 16384)])
def test_tiny_parity_options(tiny, cap_p, hop_budget, hash_cap):
    """Candidate capacity, hop budget, and a tiny LDS hash that forces the
    exact global-bitmap spill path."""
    w, gix, oix, _ = tiny
    n = 80
    Q, l, r = w["Q"][:n], w["l"][:n], w["r"][:n]
    out = gpu_search(gix, Q, l, r, 10, 64, visited_cap=4096, cand_cap=cap_p,
                     hop_budget=hop_budget, hash_cap=hash_cap)
    check_against_oracle(w, oix, out, Q, l, r, 10, 64, cap_p=cap_p, hop_budget=hop_budget)


def test_tiny_edge_ranges(tiny):
    """Single points, whole range, tree-node ranges, leaf-only ranges,
    ranges shorter than k (padding) and invalid ranges (counted, -1/+inf)."""
    w, gix, oix, _ = tiny
    n = oix.n
    rng = np.random.default_rng(9)
    L, R = [], []
    for a in (0, 1, 4999, 5000, 9998, 9999):
        L.append(a); R.append(a)                      # single point
    L += [0, 0, 5000, 0, 9990, 2500, 7, 1234, 0, 4999]
    R += [n - 1, 4999, 9999, 9, 9999, 7499, 7 + 5, 1234 + 127, 127, 5000]
    for _ in range(20):
        a = int(rng.integers(0, n)); L.append(a); R.append(min(n - 1, a + int(rng.integers(0, 40))))
    valid = len(L)
    L += [5, -1, 0, 10]
    R += [4, 3, n, n + 5]
    L = np.array(L, np.int64)
    R = np.array(R, np.int64)
    Q = w["Q"][rng.integers(0, len(w["Q"]), len(L))]
    out = gpu_search(gix, Q, L, R, 10, 64, visited_cap=4096)
    assert out["n_invalid"] == 4
    assert np.all(out["ids"][valid:] == -1) and np.all(np.isinf(out["dists"][valid:]))
    assert np.all(out["trace"]["kind"][valid:] == 0)
    check_against_oracle(w, oix, {**out, "ids": out["ids"][:valid], "dists": out["dists"][:valid],
                                  "trace": {k_: v[:valid] for k_, v in out["trace"].items()},
                                  "visited": out["visited"][:valid]},
                         Q[:valid], L[:valid], R[:valid], 10, 64)
    # ranges shorter than k are padded
    short = (R[:valid] - L[:valid] + 1) < 10
    for i in np.flatnonzero(short):
        w_ = R[i] - L[i] + 1
        assert np.all(out["ids"][i, w_:] == -1) and np.all(out["ids"][i, :w_] >= 0)


def test_tiny_bf16_fp8_traversal(tiny):
    """bfloat16 and fp8 traversal (with and without the float32 rerank)
    against the oracle running the same search on its own encodings; the
    device encodings equal the oracle's codecs."""
    w, gix, oix, path = tiny
    gix.add_storage("bf16")
    gix.add_storage("fp8")
    torch.cuda.synchronize()
    b16 = gix.copy_storage("bf16")
    codes, scale = gix.copy_storage("fp8")
    o16 = oracle.read_index(path).with_bf16()
    o8 = oracle.read_index(path).with_fp8()
    assert np.array_equal(b16, o16.vec16), "bfloat16 encodings differ"
    assert np.array_equal(scale.view(np.uint32), o8.scale8.view(np.uint32)), "fp8 scales differ"
    assert np.array_equal(codes, o8.vec8), "fp8 codes differ"
    n = 100
    Q, l, r = w["Q"][:n], w["l"][:n], w["r"][:n]
    for trav, kind, oi in (("bf16", oracle.DIST_BF16, o16), ("fp8", oracle.DIST_FP8, o8)):
        for rer in (0, 1):
            out = gpu_search(gix, Q, l, r, 10, 64, visited_cap=4096, traversal=trav, rerank=rer)
            check_against_oracle(w, oi, out, Q, l, r, 10, 64, kind=kind, rerank=rer)


@pytest.mark.parametrize("k,ef,trav", [(10, 64, "f32"), (10, 200, "f32"), (16, 512, "f32"),
                                       (10, 64, "bf16"), (10, 128, "fp8")])
def test_degree32_parity(tiny32, k, ef, trav):
    """Degree-32 graphs: expansions of up to 32 neighbours."""
    w, gix, oix, path = tiny32
    kind = {"f32": oracle.DIST_F32, "bf16": oracle.DIST_BF16, "fp8": oracle.DIST_FP8}[trav]
    oi = oix
    if trav != "f32":
        gix.add_storage(trav)
        oi = oracle.read_index(path)
        oi = oi.with_bf16() if trav == "bf16" else oi.with_fp8()
    Q, l, r = w["Q"], w["l"], w["r"]
    out = gpu_search(gix, Q, l, r, k, ef, visited_cap=8192, traversal=trav, rerank=trav != "f32")
    check_against_oracle(w, oi, out, Q, l, r, k, ef, kind=kind, rerank=int(trav != "f32"))


@pytest.mark.parametrize("k,ef,trav", [(100, 128, "f32"), (100, 128, "bf16"), (100, 128, "fp8"),
                                       (100, 256, "fp8"), (10, 64, "bf16")])
def test_embedding_parity(emb, k, ef, trav):
    """d = 768 (three, two and one 16-byte chunks per lane for float32,
    bfloat16, fp8), k = 100, with the float32 rerank for narrow storage."""
    w, gix, oix, path = emb
    kind = {"f32": oracle.DIST_F32, "bf16": oracle.DIST_BF16, "fp8": oracle.DIST_FP8}[trav]
    oi = oix
    if trav != "f32":
        gix.add_storage(trav)
        oi = oracle.read_index(path)
        oi = oi.with_bf16() if trav == "bf16" else oi.with_fp8()
    Q, l, r = w["Q"], w["l"], w["r"]
    out = gpu_search(gix, Q, l, r, k, ef, visited_cap=8192, traversal=trav, rerank=trav != "f32")
    check_against_oracle(w, oi, out, Q, l, r, k, ef, kind=kind, rerank=int(trav != "f32"))


def test_deterministic_repeat(tiny):
    w, gix, oix, _ = tiny
    a = gpu_search(gix, w["Q"], w["l"], w["r"], 10, 64)
    b = gpu_search(gix, w["Q"], w["l"], w["r"], 10, 64)
    assert np.array_equal(a["ids"], b["ids"]) and np.array_equal(a["dists"], b["dists"])


def test_argument_errors(tiny):
    w, gix, oix, _ = tiny
    Q, l, r = _t(w["Q"][:4]), _t(w["l"][:4]), _t(w["r"][:4])
    for k, ef in ((0, 10), (11, 10), (10, 1025)):
        with pytest.raises(esg.EsgError) as e:
            gix.search_ex(Q, l, r, k, ef)
        assert e.value.status == esg.ESG_EINVAL
    with pytest.raises(esg.EsgError) as e:
        gix.search_ex(Q, l, r, 10, 64, hash_cap=100)
    assert e.value.status == esg.ESG_EINVAL
    with pytest.raises(esg.EsgError) as e:
        gix.search_ex(Q, l, r, 10, 64, hash_cap=32768)
    assert e.value.status == esg.ESG_EINVAL


@pytest.mark.parametrize("nq", [0, 1, 3, 65])
def test_empty_and_ragged_batches(tiny, nq):
    """Batches of 0, 1, 3 and 65 queries (not multiples of the 4 waves of a
    workgroup): plain search, bfloat16 search replayed from a hipGraph, and
    the exact scan at its largest k (128), each against the oracle."""
    from test_gpu_scan import oracle_scan
    w, gix, oix, path = tiny
    gix.add_storage("bf16")
    gix.reserve(256, 4096)
    o16 = oracle.read_index(path).with_bf16()
    Q, l, r = w["Q"][:nq], w["l"][:nq], w["r"][:nq]
    for kw, oi, kind, rer in (({}, oix, oracle.DIST_F32, 0),
                              ({"use_graph": True, "traversal": "bf16", "rerank": True}, o16,
                               oracle.DIST_BF16, 1)):
        print(f"[gpu] ragged nq={nq} {kw}", flush=True)
        ids, dists = gix.search_ex(_t(Q), _t(l), _t(r), 10, 64, **kw)
        torch.cuda.synchronize()
        assert ids.shape == (nq, 10)
        if nq:
            oid, od, st = oracle.query_batch(oi, Q, l, r, 10, 64, 64, -1, kind, rer)
            assert np.all(st == 0)
            assert np.array_equal(ids.cpu().numpy(), oid)
            assert np.array_equal(dists.cpu().numpy().view(np.uint32), od.view(np.uint32))
    ids, dists, nfb = gix.scan(_t(Q), _t(l), _t(r), 128)
    torch.cuda.synchronize()
    assert ids.shape == (nq, 128)
    if nq:
        oid, od = oracle_scan(oix, Q, l, r, 128)
        assert np.array_equal(ids.cpu().numpy(), oid)
        assert np.array_equal(dists.cpu().numpy().view(np.uint32), od.view(np.uint32))
