"""The device builder writes the host builder's file, byte for byte.

Both run the insertion rounds of Alg. 3 (and of the half-bounded chains,
Alg. 2) with the same batches, entry points, float32 distances and
(distance, position) order; the device runs each round's beam searches,
occlusion pruning and reverse edges in kernels.  Checked on the tiny
workload (fanout 2 and 4, the chain layout, the inner-product metric at
d = 33), DEEP-shaped rows at d = 96 with a leaf of 1,024 and larger
batches, and embedding-shaped rows at d = 768.
"""
from __future__ import annotations

import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2504_04018_amd as esg  # noqa: E402

CASES = [
    ("tiny-f2", 0, 10000, None, dict(degree=16, leaf=128, ef_construction=200)),
    ("tiny-f4", 0, 10000, None, dict(degree=16, leaf=128, ef_construction=200, fanout=4)),
    ("tiny-chain", 0, 10000, None, dict(degree=16, leaf=128, ef_construction=200, layout="chain")),
    ("tiny-ip", 0, 10000, None, dict(degree=16, leaf=128, ef_construction=200, metric="ip")),
    ("deep-d96", 2, 30000, None, dict(degree=16, leaf=1024, ef_construction=200, batch_max=4096)),
    ("emb-d768", 3, 5000, None, dict(degree=16, leaf=512, ef_construction=100)),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_gpu_build_equals_host_build(case, tmp_path):
    name, cid, n, d, kw = case
    w = synth.make_workload(cid, n=n, nq=0, d=d)
    X = w["X"]
    if kw.get("metric") == "ip":
        X = synth.spread_norms(X, 0.5, 5)
    attr = w["attr"].astype(np.float64)
    ph, pg = str(tmp_path / "host.esgi"), str(tmp_path / "gpu.esgi")
    t0 = time.time()
    esg.build_index(X, attr, ph, **kw)
    t1 = time.time()
    print(f"[gpu] build {name} n={n} on the device", flush=True)
    esg.build_index(X, attr, pg, device=0, **kw)
    t2 = time.time()
    print(f"{name}: host {t1 - t0:.2f} s, device {t2 - t1:.2f} s")
    a, b = open(ph, "rb").read(), open(pg, "rb").read()
    assert len(a) == len(b)
    if a != b:
        diff = np.flatnonzero(np.frombuffer(a, np.uint8) != np.frombuffer(b, np.uint8))
        raise AssertionError(f"{len(diff)} bytes differ, first at offset {diff[0]}")


def test_gpu_build_rejects_bad_arguments(tmp_path):
    X = np.ones((100, 32), np.float32)
    with pytest.raises(esg.EsgError) as e:
        esg.build_index(X, np.arange(100.0), str(tmp_path / "x"), device=0, batch_max=8193)
    assert e.value.status == esg.ESG_EINVAL
    with pytest.raises(esg.EsgError) as e:
        esg.build_index(np.ones((100, 8), np.float32), np.arange(100.0), str(tmp_path / "y"),
                        leaf=16, device=0)
    assert e.value.status == esg.ESG_EUNSUPPORTED
