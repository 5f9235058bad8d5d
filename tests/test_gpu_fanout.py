"""GPU parity on fanout-f indexes (Section 4.2, Extensions; Lemma 4.3).

The tiny workload (N = 10,000, d = 32, leaf 128, degree 16) built with
fanout 4 and 16 (elastic constant 1/f): for every query the GPU's parts
(tree node, node number, range piece), visited sets, hop counts, ids and
float32 distances equal the oracle's, for float32 and bfloat16 traversal,
with the learned switch too; graph memory shrinks with the fanout.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import tree_nodes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2504_04018_amd as esg  # noqa: E402
from tests.test_gpu_search import check_against_oracle, gpu_search  # noqa: E402

DEV = torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module", params=[4, 16], ids=lambda f: f"f{f}")
def fan(request, tmp_path_factory):
    f = request.param
    w = synth.make_workload(0, nq=300)
    path = str(tmp_path_factory.mktemp(f"fan{f}") / "tiny.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=16, leaf=w["leaf"],
                    ef_construction=200, fanout=f)
    gix = esg.Index(path, 0)
    oix = oracle.read_index(path)
    # more narrow ranges than the workload's law: they reach the deep levels
    rng = np.random.default_rng(f)
    wd = np.rint(np.exp(rng.uniform(0, np.log(w["n"]), 300))).astype(np.int64)
    l = (rng.random(300) * (w["n"] - wd + 1)).astype(np.int64)
    w["l"], w["r"] = l, l + wd - 1
    yield w, gix, oix, f
    gix.free()


def test_fanout_index_shape(fan):
    w, gix, oix, f = fan
    info = gix.info()
    assert info["fanout"] == f and info["c_den"] == f
    depths = {t for t, _, _, _, g in tree_nodes(oix.n, oix.leaf, f) if g}
    assert info["n_depth"] == len(depths) == {4: 4, 16: 2}[f]


@pytest.mark.parametrize("trav", ["f32", "bf16"])
def test_fanout_parity(fan, trav):
    w, gix, oix, f = fan
    Q, l, r = w["Q"], w["l"], w["r"]
    kind = oracle.DIST_F32
    if trav == "bf16":
        gix.add_storage("bf16")
        oix = oracle.read_index(gix.path).with_bf16()
        kind = oracle.DIST_BF16
    out = gpu_search(gix, Q, l, r, 10, 64, visited_cap=4096, traversal=trav,
                     rerank=trav != "f32")
    check_against_oracle(w, oix, out, Q, l, r, 10, 64, kind=kind, rerank=int(trav != "f32"))
    tr = out["trace"]
    n_parts = (tr["kind"] > 0).sum(1)
    assert n_parts.max() == 2 and n_parts.min() == 1
    # every node depth of the tree is reached by some graph part
    assert set(tr["depth"][tr["kind"] == 1].tolist()) == set(range(oix.n_depth))


def test_fanout_learned_parity(fan):
    """The learned beam width on a fanout-f tree: features equal the
    oracle's, and with the GPU's beams the oracle reproduces the answers."""
    w, gix, oix, f = fan
    Q, l, r = w["Q"], w["l"], w["r"]
    nq, k, ef, probe = len(Q), 10, 64, 4
    rng = np.random.default_rng(30 + f)
    p = np.concatenate([rng.standard_normal(5057) * 0.15, rng.standard_normal(12),
                        np.abs(rng.standard_normal(12)) + 0.5]).astype(np.float32)
    p[5057:5069] = [8, 9, 0.5, 9, 0.5, 0.5, 2, 0.5, 0.5, 1, 1, 7]
    p[5069:] = [3, 3, 0.3, 3, 0.5, 0.3, 1.5, 0.3, 0.3, 0.5, 0.5, 2]
    p[5056] = 4.5
    feat = torch.full((nq, 2, 16), float("nan"), device=DEV)
    print(f"[gpu] fanout {f} learned", flush=True)
    ids, dists = gix.search_ex(_t(Q), _t(l), _t(r), k, ef, mlp=_t(p), probe_hops=probe,
                               feat_out=feat)
    torch.cuda.synchronize()
    F, ids, dists = feat.cpu().numpy(), ids.cpu().numpy(), dists.cpu().numpy()
    switched = 0
    for i in range(nq):
        parts, npart = oix.select(l[i], r[i])
        ef2 = np.zeros(2, np.int32)
        for j, pt in enumerate(parts):
            if pt["kind"] != oracle.KIND_GRAPH:
                continue
            _, _, _, _, _, f64 = oracle.search_part_learned(
                oix, pt, Q[i], ef, probe, 0, k, int(r[i] - l[i] + 1), npart)
            assert np.isnan(F[i, j, 0]) == (f64 is None), (i, j)
            if f64 is None:
                continue
            switched += 1
            assert np.allclose(F[i, j, :12], f64, rtol=1e-4, atol=1e-5), (i, j)
            ef2[j] = int(F[i, j, 13])
        oid, od, _, st = oracle.query_learned(oix, Q[i], int(l[i]), int(r[i]), k, ef, probe, ef2)
        assert st == 0
        assert np.array_equal(ids[i], oid), i
        assert np.array_equal(dists[i].view(np.uint32), od.view(np.uint32)), i
    assert switched > 50
