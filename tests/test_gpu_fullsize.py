"""GPU parity at the bench's full size: the DEEP-shaped set (N = 1,000,000,
d = 96, R = 32, leaf 1,024) and its whole batch of 100,000 queries in one
launch, as bench.py times it, the SIFT-shaped set (1M x 128) and the
embedding-shaped set (2M x 768, k = 100); sampled outputs are checked one by one
against the oracle (bit-exact ids and float32 distances).  The indexes are
built on the device, as the bench builds them (the host builder writes the
same file: test_gpu_build)."""
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

DEV = torch.device("cuda:0")
SAMPLE = 64


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def deep(tmp_path_factory):
    w = synth.make_workload(2)
    path = str(tmp_path_factory.mktemp("deep") / "deep1M.esgi")
    print("[gpu] building the 1M x 96 index on the device", flush=True)
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=w["degree"],
                    leaf=w["leaf"], ef_construction=w["ef_construction"], device=0)
    del w["X"]
    gix = esg.Index(path, 0)
    gix.add_storage("bf16")
    yield w, gix, path
    gix.free()


def _sample(nq, seed):
    return np.sort(np.random.default_rng(seed).choice(nq, SAMPLE, replace=False))


@pytest.mark.parametrize("trav,ef", [("f32", 22), ("bf16", 22)])
def test_full_batch_sampled_parity(deep, trav, ef):
    w, gix, path = deep
    Q, l, r = w["Q"], w["l"], w["r"]
    print(f"[gpu] full batch {len(Q)} queries {trav} ef={ef}", flush=True)
    ids, dists = gix.search_ex(_t(Q), _t(l), _t(r), 10, ef, traversal=trav,
                               rerank=trav != "f32")
    torch.cuda.synchronize()
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    oix = oracle.read_index(path)
    kind = oracle.DIST_F32
    if trav == "bf16":
        oix = oix.with_bf16()
        kind = oracle.DIST_BF16
    s = _sample(len(Q), 7 if trav == "f32" else 8)
    oid, od, st = oracle.query_batch(oix, Q[s], l[s], r[s], 10, ef, ef, -1, kind,
                                     int(trav != "f32"))
    assert np.all(st == 0)
    assert np.array_equal(ids[s], oid)
    assert np.array_equal(dists[s].view(np.uint32), od.view(np.uint32))


def test_full_batch_learned_sampled_parity(deep):
    """The learned kernel over the whole batch (probe 4 hops at ef 32): the
    oracle, given the beams the GPU chose, reproduces the sampled answers."""
    w, gix, path = deep
    Q, l, r = w["Q"], w["l"], w["r"]
    nq = len(Q)
    rng = np.random.default_rng(3)
    p = np.concatenate([rng.standard_normal(5057) * 0.15, rng.standard_normal(12),
                        np.abs(rng.standard_normal(12)) + 0.5]).astype(np.float32)
    p[5056] = 4.0                                      # log2 beam around 4
    feat = torch.full((nq, 2, 16), float("nan"), device=DEV)
    print("[gpu] full batch learned", flush=True)
    ids, dists = gix.search_ex(_t(Q), _t(l), _t(r), 10, 32, mlp=_t(p), probe_hops=4,
                               feat_out=feat)
    torch.cuda.synchronize()
    ids, dists, F = ids.cpu().numpy(), dists.cpu().numpy(), feat.cpu().numpy()
    oix = oracle.read_index(path)
    switched = 0
    for i in _sample(nq, 9):
        ef2 = np.zeros(2, np.int32)
        for j in range(2):
            if not np.isnan(F[i, j, 0]):
                ef2[j] = int(F[i, j, 13])
                switched += 1
        oid, od, _, st = oracle.query_learned(oix, Q[i], int(l[i]), int(r[i]), 10, 32, 4, ef2)
        assert st == 0
        assert np.array_equal(ids[i], oid), i
        assert np.array_equal(dists[i].view(np.uint32), od.view(np.uint32)), i
    assert switched > SAMPLE // 2


def test_full_batch_learned_before_search_sampled_parity(deep):
    """The learned form the bench times (beams chosen before the search,
    bfloat16 traversal + float32 rerank, ef cap 32) over the whole batch:
    given the GPU's per-part beams, the oracle (its switch at hop 0)
    reproduces the sampled answers bit for bit."""
    w, gix, path = deep
    Q, l, r = w["Q"], w["l"], w["r"]
    nq = len(Q)
    gix.reserve(nq, 262144)
    rng = np.random.default_rng(13)
    p = np.concatenate([rng.standard_normal(5056) * 0.15, [4.3],
                        [14, 15, 0.6, 14, 0.3] + [0.0] * 7,          # feature means
                        [3, 3, 0.3, 3, 0.5] + [1e-3] * 7]).astype(np.float32)
    feat = torch.full((nq, 2, 16), float("nan"), device=DEV)
    print("[gpu] full batch learned, beams before the search", flush=True)
    ids, dists = gix.search_ex(_t(Q), _t(l), _t(r), 10, 32, traversal="bf16", rerank=True,
                               mlp=_t(p), probe_hops=0, feat_out=feat)
    torch.cuda.synchronize()
    ids, dists, F = ids.cpu().numpy(), dists.cpu().numpy(), feat.cpu().numpy()
    oix = oracle.read_index(path).with_bf16()
    beams = set()
    for i in _sample(nq, 14):
        ef2 = np.where(np.isnan(F[i, :, 13]), 0, F[i, :, 13]).astype(np.int32)
        beams.update(int(v) for v in ef2 if v > 0)
        oid, od, _, st = oracle.query_learned(oix, Q[i], int(l[i]), int(r[i]), 10, 32, 0, ef2,
                                              kind=oracle.DIST_BF16, rerank=1)
        assert st == 0
        assert np.array_equal(ids[i], oid), i
        assert np.array_equal(dists[i].view(np.uint32), od.view(np.uint32)), i
    assert len(beams) > 3


def test_full_batch_scan_sampled(deep):
    """The exact scan over the whole 100,000-query batch, as the bench runs it
    for its recall reference: 64 sampled queries equal the oracle's float32 scan
    bit for bit, and their top 10 agree with the float64 brute force of
    Def. 2.2 (every returned point lies within the 10th exact distance)."""
    w, gix, path = deep
    Q, l, r = w["Q"], w["l"], w["r"]
    nq = len(Q)
    gix.reserve(nq, 262144)
    print("[gpu] full batch exact scan", flush=True)
    ids, dists, nfb = gix.scan(_t(Q), _t(l), _t(r), 10)
    torch.cuda.synchronize()
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    oix = oracle.read_index(path)
    s = _sample(nq, 10)
    oid, od = oracle_scan(oix, Q[s], l[s], r[s], 10)
    assert np.array_equal(ids[s], oid)
    assert np.array_equal(dists[s].view(np.uint32), od.view(np.uint32))
    pos_of = np.empty(oix.n, np.int64)
    pos_of[oix.ext_id] = np.arange(oix.n)
    found = np.where(ids[s] >= 0, pos_of[np.maximum(ids[s], 0)], -1)
    gt_pos, gt_d = oracle.bruteforce(oix.vec, Q[s], l[s], r[s], 10)
    rec, strict, _ = oracle.recall(oix.vec, Q[s], l[s], r[s], found, gt_pos, gt_d, 10)
    print(f"scan vs float64 brute force: recall {rec}, strict {strict}, rescans {nfb}")
    assert rec == 1.0


@pytest.fixture(scope="module")
def sift(tmp_path_factory):
    w = synth.make_workload(1)
    path = str(tmp_path_factory.mktemp("sift") / "sift1M.esgi")
    print("[gpu] building the 1M x 128 index on the device", flush=True)
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=w["degree"],
                    leaf=w["leaf"], ef_construction=w["ef_construction"], device=0)
    del w["X"]
    return w, path


@pytest.mark.parametrize("trav", ["f32", "bf16"])
def test_sift_full_size_sampled_parity(sift, trav):
    """SIFT-shaped at full size (N = 1M, d = 128 uint8-valued, the 10,000
    queries of 11 width buckets in one launch, ef 64): sampled queries
    bit-exact against the oracle."""
    w, path = sift
    gix = esg.Index(path, 0)
    if trav == "bf16":
        gix.add_storage("bf16")
    Q, l, r = w["Q"], w["l"], w["r"]
    print(f"[gpu] sift full batch {trav}", flush=True)
    ids, dists = gix.search_ex(_t(Q), _t(l), _t(r), 10, 64, traversal=trav,
                               rerank=trav != "f32")
    torch.cuda.synchronize()
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    gix.free()
    oix = oracle.read_index(path)
    kind = oracle.DIST_F32
    if trav == "bf16":
        oix = oix.with_bf16()
        kind = oracle.DIST_BF16
    s = _sample(len(Q), 11)
    oid, od, st = oracle.query_batch(oix, Q[s], l[s], r[s], 10, 64, 64, -1, kind,
                                     int(trav != "f32"))
    assert np.all(st == 0)
    assert np.array_equal(ids[s], oid)
    assert np.array_equal(dists[s].view(np.uint32), od.view(np.uint32))


@pytest.fixture(scope="module")
def embedding(tmp_path_factory):
    """The embedding-shaped set at full size (N = 2,000,000, d = 768, R = 32,
    leaf 1,024; 20,000 queries in 13 width buckets, k = 100)."""
    w = synth.make_workload(3)
    path = str(tmp_path_factory.mktemp("emb") / "emb2M.esgi")
    print("[gpu] building the 2M x 768 index on the device", flush=True)
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=w["degree"],
                    leaf=w["leaf"], ef_construction=w["ef_construction"], device=0)
    del w["X"]
    gix = esg.Index(path, 0)
    yield w, gix, path
    gix.free()


def test_embedding_full_size_sampled_parity(embedding):
    """The 20,000-query batch in one launch (float32 traversal, k = 100, ef
    112, the bench's calibrated beam): 16 sampled queries bit-exact against
    the oracle; and the exact scan (k = 100) on 8 sampled queries equal to
    the oracle's float32 scan."""
    w, gix, path = embedding
    Q, l, r = w["Q"], w["l"], w["r"]
    nq, k = len(Q), w["k"]
    print(f"[gpu] embedding full batch {nq} queries k={k} ef=112", flush=True)
    ids, dists = gix.search_ex(_t(Q), _t(l), _t(r), k, 112)
    torch.cuda.synchronize()
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    oix = oracle.read_index(path)
    s = np.sort(np.random.default_rng(11).choice(nq, 16, replace=False))
    oid, od, st = oracle.query_batch(oix, Q[s], l[s], r[s], k, 112)
    assert np.all(st == 0)
    assert np.array_equal(ids[s], oid)
    assert np.array_equal(dists[s].view(np.uint32), od.view(np.uint32))
    gix.add_storage("bf16")
    gix.reserve(nq, 4_500_000)
    print("[gpu] embedding exact scan", flush=True)
    sids, sd, nfb = gix.scan(_t(Q), _t(l), _t(r), k)
    torch.cuda.synchronize()
    s = np.sort(np.random.default_rng(12).choice(nq, 8, replace=False))
    oid, od = oracle_scan(oix, Q[s], l[s], r[s], k)
    assert np.array_equal(sids.cpu().numpy()[s], oid)
    assert np.array_equal(sd.cpu().numpy()[s].view(np.uint32), od.view(np.uint32))
