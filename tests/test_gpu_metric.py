"""GPU parity and recall of inner-product and angular indexes, and of
dimensions served by a wider kernel class.

Inner product and angular distance are reduced to squared Euclidean
distance when the index is built (unit rows; the one-coordinate transform
of Bachrach et al., RecSys 2014, which stores d + 1 values and reads a
query's d values followed by a 0): the paper's search then runs unchanged
(it leaves these metrics open, Section 7).  On the tiny workload with
log-normally spread norms: the GPU's parts, visited sets, hops, ids and
float32 distances equal the oracle's for float32 and bfloat16 traversal
and for the brute-force scan; the answers reach the exact top 10 of the
metric; and the inner product recovered from a returned distance matches
the float64 one.  Kernels compiled for one dimension serve every
dimension with the same lane shape: d = 100 (GLOVE-shaped, class 128),
1024 and 2048 (WIT-shaped) also match the oracle.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import oracle_scan

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2504_04018_amd as esg  # noqa: E402
from tests.test_gpu_search import check_against_oracle, gpu_search  # noqa: E402

DEV = torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module", params=["ip", "angular"])
def midx(request, tmp_path_factory):
    m = request.param
    w = synth.make_workload(0, nq=300)
    X = synth.spread_norms(w["X"], 0.5, 21)
    path = str(tmp_path_factory.mktemp(f"metric_{m}") / "tiny.esgi")
    esg.build_index(X, w["attr"].astype(np.float64), path, degree=16, leaf=w["leaf"],
                    ef_construction=200, metric=m)
    gix = esg.Index(path, 0)
    oix = oracle.read_index(path)
    assert gix.metric == m and gix.dq == 32 and gix.d == (33 if m == "ip" else 32)
    yield w, X, gix, oix, {"ip": oracle.METRIC_IP, "angular": oracle.METRIC_ANGULAR}[m]
    gix.free()


@pytest.mark.parametrize("trav", ["f32", "bf16"])
def test_metric_parity(midx, trav):
    w, X, gix, oix, metric = midx
    Q, l, r = w["Q"], w["l"], w["r"]
    kind = oracle.DIST_F32
    if trav == "bf16":
        gix.add_storage("bf16")
        oix = oracle.read_index(gix.path).with_bf16()
        kind = oracle.DIST_BF16
    out = gpu_search(gix, Q, l, r, 10, 64, visited_cap=4096, traversal=trav,
                     rerank=trav != "f32")
    check_against_oracle(w, oix, out, Q, l, r, 10, 64, kind=kind, rerank=int(trav != "f32"))


def test_metric_scan_parity(midx):
    w, X, gix, oix, metric = midx
    Q, l, r = w["Q"], w["l"], w["r"]
    gix.add_storage("bf16")
    gix.reserve(len(Q), 4096)
    print(f"[gpu] metric {gix.metric} scan", flush=True)
    ids, dists, nfb = gix.scan(_t(Q), _t(l), _t(r), 10)
    torch.cuda.synchronize()
    oid, od = oracle_scan(oix, Q, l, r, 10)
    assert np.array_equal(ids.cpu().numpy(), oid)
    assert np.array_equal(dists.cpu().numpy().view(np.uint32), od.view(np.uint32))


def test_metric_recall_and_scores(midx):
    """Recall of the metric's exact top 10 (float64, original rows) and,
    for inner product, <x, q> = (M^2 + |q|^2 - dist) / 2 within float32
    rounding of the stored-space distance."""
    w, X, gix, oix, metric = midx
    Q, l, r = w["Q"], w["l"], w["r"]
    print(f"[gpu] metric {gix.metric} recall", flush=True)
    ids, dists = gix.search_ex(_t(Q), _t(l), _t(r), 10, 64)
    torch.cuda.synchronize()
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    gt, score = oracle.exact_metric(X[oix.ext_id], Q, l, r, 10, metric)
    pos_of = np.empty(oix.n, np.int64)
    pos_of[oix.ext_id] = np.arange(oix.n)
    hit = tot = 0
    for i in range(len(Q)):
        g = gt[i][gt[i] >= 0]
        f = pos_of[ids[i][ids[i] >= 0]]
        hit += len(np.intersect1d(g, f))
        tot += len(g)
    print(f"{gix.metric}: recall@10 {hit / tot:.4f}")
    assert hit / tot >= 0.95
    if metric == oracle.METRIC_IP:
        ok = ids >= 0
        q2 = np.sum(Q.astype(np.float64) ** 2, axis=1)[:, None]
        ip_gpu = (gix.max_norm2 + q2 - dists.astype(np.float64)) / 2
        ip64 = np.einsum("ikd,id->ik", X[np.maximum(ids, 0)].astype(np.float64),
                         Q.astype(np.float64))
        scale = gix.max_norm2 + q2
        assert np.all(np.abs(ip_gpu - ip64)[ok] <= (1e-5 * np.broadcast_to(scale, ok.shape))[ok])


@pytest.fixture(scope="module", params=[(2, 100), (3, 1024), (3, 2048)],
                ids=lambda p: f"d{p[1]}")
def wide(request, tmp_path_factory):
    cid, d = request.param
    w = synth.make_workload(cid, n=4000, nq=100, d=d)
    path = str(tmp_path_factory.mktemp(f"wide{d}") / "w.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=16, leaf=128,
                    ef_construction=64)
    gix = esg.Index(path, 0)
    oix = oracle.read_index(path)
    rng = np.random.default_rng(d)
    wd = np.rint(np.exp(rng.uniform(0, np.log(4000), 100))).astype(np.int64)
    l = (rng.random(100) * (4000 - wd + 1)).astype(np.int64)
    w["l"], w["r"] = l, l + wd - 1
    yield w, gix, oix
    gix.free()


@pytest.mark.parametrize("trav", ["f32", "bf16"])
def test_class_dims_parity(wide, trav):
    w, gix, oix = wide
    Q, l, r = w["Q"], w["l"], w["r"]
    kind = oracle.DIST_F32
    if trav == "bf16":
        gix.add_storage("bf16")
        oix = oracle.read_index(gix.path).with_bf16()
        kind = oracle.DIST_BF16
    out = gpu_search(gix, Q, l, r, 10, 64, visited_cap=4096, traversal=trav,
                     rerank=trav != "f32")
    check_against_oracle(w, oix, out, Q, l, r, 10, 64, kind=kind, rerank=int(trav != "f32"))
