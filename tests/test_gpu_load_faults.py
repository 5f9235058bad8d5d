"""Failure handling of the index loader, forced from the host.

Each case runs one load in a child process with a test hook set (the hooks
count events per process):
  * ESG_FAULT_ALLOC_AT=n: the n-th device allocation fails; the load
    reports ESG_ENOMEM and releases what it took;
  * ESG_FAULT_UPLOAD_CHECK=1: the first comparison of a device copy with
    the file reports a difference; the loader copies again and succeeds;
  * ESG_FAULT_UPLOAD_CHECK=all: every comparison reports a difference; the
    load fails with ESG_EHIP after the second copy.
No kernel is made to fault: the conditions are decided on the host.
"""
from __future__ import annotations

import os
import subprocess
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2504_04018_amd as esg  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import paper_2504_04018_amd as esg
try:
    ix = esg.Index({path!r}, 0)
    print("LOADED", ix.n, flush=True)
    ix.free()
except esg.EsgError as e:
    print("ERROR", e, flush=True)
"""


@pytest.fixture(scope="module")
def small(tmp_path_factory):
    w = synth.make_workload(0, n=3000, nq=10)
    path = str(tmp_path_factory.mktemp("faults") / "small.esgi")
    esg.build_index(w["X"], w["attr"].astype(np.float64), path, degree=16, leaf=100,
                    ef_construction=64)
    return path


def _load_in_child(path, **hooks):
    env = dict(os.environ)
    env.pop("ESG_FAULT_ALLOC_AT", None)
    env.pop("ESG_FAULT_UPLOAD_CHECK", None)
    env.update({k: str(v) for k, v in hooks.items()})
    print(f"child load of {path} with {hooks}", flush=True)
    p = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, path=path)], env=env,
                       capture_output=True, text=True, timeout=180)
    assert p.returncode == 0, p.stderr[-2000:]
    return p.stdout, p.stderr


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_allocation_failure_reports_enomem(small, n):
    out, _ = _load_in_child(small, ESG_FAULT_ALLOC_AT=n)
    assert "ERROR" in out and "ESG_ENOMEM" in out, out


def test_allocations_past_the_load_do_not_fail_it(small):
    out, _ = _load_in_child(small, ESG_FAULT_ALLOC_AT=1000)
    assert "LOADED 3000" in out, out


def test_upload_check_difference_is_copied_again(small):
    out, err = _load_in_child(small, ESG_FAULT_UPLOAD_CHECK=1)
    assert "LOADED 3000" in out, out
    assert "differs from the file; copying again" in err, err


def test_upload_check_persistent_difference_fails(small):
    out, err = _load_in_child(small, ESG_FAULT_UPLOAD_CHECK="all")
    assert "ERROR" in out and "ESG_EHIP" in out, out
    assert "differs again" in err, err


def test_load_without_hooks_still_works(small):
    ix = esg.Index(small, 0)
    assert ix.n == 3000
    ix.free()
