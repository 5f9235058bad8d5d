"""GPU parity on the half-bounded index (Section 4.1, Alg. 2, Lemma 4.1).

The tiny workload (N = 10,000, d = 32, leaf 128, degree 16) built as
prefix and suffix chains with base 2 and 4: for prefix, suffix and general
ranges the GPU's part (recorded range, depth, node number), visited set,
hop count, ids and float32 distances equal the oracle's, for float32 and
bfloat16 traversal; graph memory is O(N).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2504_04018_amd as esg  # noqa: E402
from tests.test_gpu_search import check_against_oracle, gpu_search  # noqa: E402

NQ = 300


@pytest.fixture(scope="module", params=[2, 4], ids=lambda b: f"B{b}")
def chain(request, tmp_path_factory):
    B = request.param
    w = synth.make_workload(0, nq=NQ)
    path = str(tmp_path_factory.mktemp(f"chain{B}") / "tiny.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=16, leaf=w["leaf"],
                    ef_construction=200, fanout=B, layout="chain")
    gix = esg.Index(path, 0)
    oix = oracle.read_index(path)
    n = w["n"]
    rng = np.random.default_rng(40 + B)
    wd = np.clip(np.rint(np.exp(rng.uniform(0, np.log(n), NQ))).astype(np.int64), 1, n)
    kind = np.arange(NQ) % 3                 # 0 prefix, 1 suffix, 2 general
    l = np.where(kind == 0, 0, np.where(kind == 1, n - wd, (rng.random(NQ) * (n - wd + 1)).astype(np.int64)))
    w["l"], w["r"] = l, l + wd - 1
    yield w, gix, oix, B
    gix.free()


def test_chain_index_shape(chain):
    w, gix, oix, B = chain
    info = gix.info()
    sizes, _ = oracle.chain_levels(oix.n, oix.leaf, B)
    assert info["n_depth"] == len(sizes) and info["fanout"] == B
    # O(N) graph rows: at most 2 B/(B-1) N per chain, against N per tree depth
    assert sum(sizes) <= 2 * (2 * oix.n * B // (B - 1) + len(sizes))


@pytest.mark.parametrize("trav", ["f32", "bf16"])
def test_chain_parity(chain, trav):
    w, gix, oix, B = chain
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
    assert np.all((tr["kind"] > 0).sum(1) == 1)
    graph_depths = set(tr["depth"][:, 0][tr["kind"][:, 0] == 1].tolist())
    K = oix.n_depth // 2
    assert any(d < K for d in graph_depths) and any(d >= K for d in graph_depths)
