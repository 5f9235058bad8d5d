"""GPU parity of the MFMA brute-force scan and of the narrow-range router.

The scan's contract is exactness: its answer equals the oracle's float32
scan of [l,r] (top k by the canonical float32 distance, ties by position),
whatever the certificate decided.  The router sends queries narrower than
a threshold to the scan and the rest to the graph search; each side must
equal its oracle.  hipGraph replays must equal eager runs.
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

DEV = torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def idx(tmp_path_factory):
    """Tiny workload (N=10,000, d=32) with bfloat16 storage and a reservation."""
    w = synth.make_workload(0)
    path = str(tmp_path_factory.mktemp("scan") / "tiny.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=16, leaf=w["leaf"],
                    ef_construction=200)
    gix = esg.Index(path, 0)
    gix.add_storage("bf16")
    gix.reserve(4096, 8192)
    oix = oracle.read_index(path)
    yield w, gix, oix
    gix.free()


def mixed_ranges(n, m, seed):
    rng = np.random.default_rng(seed)
    w = np.rint(np.exp(rng.uniform(0, np.log(n), m))).astype(np.int64)
    w = np.clip(w, 1, n)
    l = (rng.random(m) * (n - w + 1)).astype(np.int64)
    return l, l + w - 1


@pytest.mark.parametrize("k", [1, 10, 32, 64, 100])
def test_scan_exact(idx, k):
    """Any width (1 .. N, several 2,048-point windows): equal to the float32 scan."""
    w, gix, oix = idx
    l, r = mixed_ranges(oix.n, 300, k)
    Q = w["Q"][np.arange(300) % len(w["Q"])]
    cert = torch.zeros(300, dtype=torch.int32, device=DEV)
    print(f"[gpu] scan k={k}", flush=True)
    ids, dists, nfb = gix.scan(_t(Q), _t(l), _t(r), k, certified=cert)
    torch.cuda.synchronize()
    oid, od = oracle_scan(oix, Q, l, r, k)
    assert np.array_equal(ids.cpu().numpy(), oid)
    assert np.array_equal(dists.cpu().numpy().view(np.uint32), od.view(np.uint32))
    c = cert.cpu().numpy()
    print(f"certified {c.mean():.3f} fallback {nfb}")
    assert nfb == int((c == 0).sum())
    assert c.mean() > 0.5


@pytest.mark.parametrize("k", [1, 10, 100])
def test_scan_forced_exact(idx, k):
    """Every query through the exact path (each window's exact top k, then a
    merge per query): equal to the float32 scan, all counted as rescans."""
    w, gix, oix = idx
    l, r = mixed_ranges(oix.n, 200, 100 + k)
    Q = w["Q"][np.arange(200) % len(w["Q"])]
    print(f"[gpu] exact scan k={k}", flush=True)
    ids, dists, nfb = gix.scan(_t(Q), _t(l), _t(r), k, exact=True)
    torch.cuda.synchronize()
    oid, od = oracle_scan(oix, Q, l, r, k)
    assert nfb == 200
    assert np.array_equal(ids.cpu().numpy(), oid)
    assert np.array_equal(dists.cpu().numpy().view(np.uint32), od.view(np.uint32))


def test_scan_invalid_and_tiny_ranges(idx):
    w, gix, oix = idx
    l = np.array([0, 5, 9999, 3, -1, 10, 0], np.int64)
    r = np.array([0, 5, 9999, 40, 4, 9, 10000], np.int64)
    Q = w["Q"][:7]
    ids, dists, nfb = gix.scan(_t(Q), _t(l), _t(r), 10)
    ids = ids.cpu().numpy()
    assert np.all(ids[4:] == -1)
    oid, od = oracle_scan(oix, Q[:4], l[:4], r[:4], 10)
    assert np.array_equal(ids[:4], oid)


@pytest.mark.parametrize("thr,trav", [(512, "f32"), (2048, "bf16"), (1, "f32")])
def test_router_parity(idx, thr, trav):
    """Queries narrower than thr: equal to the float32 scan; the others: equal
    to the oracle's graph search (Alg. 4)."""
    w, gix, oix = idx
    l, r = mixed_ranges(oix.n, 600, thr)
    Q = w["Q"][np.arange(600) % len(w["Q"])]
    k, ef = 10, 64
    print(f"[gpu] router thr={thr} {trav}", flush=True)
    ids, dists = gix.search_ex(_t(Q), _t(l), _t(r), k, ef, traversal=trav, rerank=trav != "f32",
                               router_threshold=thr)
    torch.cuda.synchronize()
    ids = ids.cpu().numpy()
    dists = dists.cpu().numpy()
    narrow = (r - l + 1) < thr
    sid, sd = oracle_scan(oix, Q[narrow], l[narrow], r[narrow], k)
    assert np.array_equal(ids[narrow], sid)
    assert np.array_equal(dists[narrow].view(np.uint32), sd.view(np.uint32))
    oi = oix if trav == "f32" else oracle.read_index(gix.path).with_bf16()
    kind = oracle.DIST_F32 if trav == "f32" else oracle.DIST_BF16
    gid, gd, st = oracle.query_batch(oi, Q[~narrow], l[~narrow], r[~narrow], k, ef, ef, -1, kind,
                                     int(trav != "f32"))
    assert np.array_equal(ids[~narrow], gid)
    assert np.array_equal(dists[~narrow].view(np.uint32), gd.view(np.uint32))


@pytest.mark.parametrize("thr", [0, 1024])
def test_graph_replay(idx, thr):
    """Captured hipGraph replays equal the eager run, with eager work between."""
    w, gix, oix = idx
    l, r = mixed_ranges(oix.n, 500, 77)
    Q = _t(w["Q"][np.arange(500) % len(w["Q"])])
    lt, rt = _t(l), _t(r)
    ref_i, ref_d = gix.search_ex(Q, lt, rt, 10, 64, router_threshold=thr)
    torch.cuda.synchronize()
    ref_i, ref_d = ref_i.clone(), ref_d.clone()
    ids = torch.empty_like(ref_i)
    dists = torch.empty_like(ref_d)
    for rep in range(4):
        ids.fill_(-7)
        dists.fill_(-7.0)
        gix.search_ex(Q, lt, rt, 10, 64, router_threshold=thr, use_graph=True, ids=ids,
                      dists=dists)
        torch.cuda.synchronize()
        assert torch.equal(ids, ref_i) and torch.equal(dists, ref_d), rep
        # unrelated eager work between replays
        gix.search_ex(Q[:50], lt[:50], rt[:50], 5, 32)
        torch.cuda.synchronize()


@pytest.mark.parametrize("probe", [1, 4])
def test_router_with_learned_beam(idx, probe):
    """Router + learned beam width + hipGraph replay: narrow queries equal the
    float32 scan; wide ones equal the same learned search run without the
    router on just those queries (the router only splits the batch)."""
    w, gix, oix = idx
    l, r = mixed_ranges(oix.n, 400, 300 + probe)
    Q = w["Q"][np.arange(400) % len(w["Q"])]
    rng = np.random.default_rng(5)
    p = np.concatenate([rng.standard_normal(5057) * 0.15, rng.standard_normal(12),
                        np.abs(rng.standard_normal(12)) + 0.5]).astype(np.float32)
    p[5056] = 4.5
    mlp = _t(p)
    k, ef, thr = 10, 64, 1024
    print(f"[gpu] router + learned probe={probe}", flush=True)
    ids, dists = gix.search_ex(_t(Q), _t(l), _t(r), k, ef, router_threshold=thr, mlp=mlp,
                               probe_hops=probe, use_graph=True)
    torch.cuda.synchronize()
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    narrow = (r - l + 1) < thr
    sid, sd = oracle_scan(oix, Q[narrow], l[narrow], r[narrow], k)
    assert np.array_equal(ids[narrow], sid)
    assert np.array_equal(dists[narrow].view(np.uint32), sd.view(np.uint32))
    wi, wd = gix.search_ex(_t(Q[~narrow]), _t(l[~narrow]), _t(r[~narrow]), k, ef, mlp=mlp,
                           probe_hops=probe)
    torch.cuda.synchronize()
    assert np.array_equal(ids[~narrow], wi.cpu().numpy())
    assert np.array_equal(dists[~narrow].view(np.uint32), wd.cpu().numpy().view(np.uint32))
