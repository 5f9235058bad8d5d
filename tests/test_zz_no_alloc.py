"""The allocation-free gradient entry point (esg_mlp_grad_noalloc) against
esg_mlp_grad, called through the C ABI: identical gradients and losses,
bit for bit, on two calls in a row, the second with a smaller batch (the
library's scratch keeps the first call's contents)."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2504_04018_amd as esg  # noqa: E402

DEV = torch.device("cuda:0")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def test_noalloc_grad_matches_workspace_grad():
    rng = np.random.default_rng(21)
    p = np.concatenate([rng.standard_normal(esg.MLP_WEIGHTS) * 0.2, rng.standard_normal(12),
                        np.abs(rng.standard_normal(12)) + 0.5]).astype(np.float32)
    P = torch.from_numpy(p).to(DEV)
    L = esg.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ws = torch.zeros(esg.MLP_WORKSPACE_FLOATS, device=DEV)
    for n in (5000, 700):
        print(f"[gpu] noalloc grad n={n}", flush=True)
        F = torch.from_numpy((rng.standard_normal((n, 12)) * 2).astype(np.float32)).to(DEV)
        T = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(DEV)
        g_ref = torch.full((esg.MLP_WEIGHTS,), float("nan"), device=DEV)
        l_ref = torch.full((1,), float("nan"), device=DEV)
        g_new = torch.full((esg.MLP_WEIGHTS,), float("nan"), device=DEV)
        l_new = torch.full((1,), float("nan"), device=DEV)
        st = L.esg_mlp_grad(_ptr(P), _ptr(F), _ptr(T), n, _ptr(g_ref), _ptr(l_ref), _ptr(ws),
                            stream)
        assert st == esg.ESG_OK
        st = L.esg_mlp_grad_noalloc(_ptr(P), _ptr(F), _ptr(T), n, _ptr(g_new), _ptr(l_new),
                                    stream)
        assert st == esg.ESG_OK
        torch.cuda.synchronize()
        assert torch.isfinite(g_ref).all() and torch.isfinite(l_ref).all()
        assert torch.equal(g_new, g_ref), n
        assert torch.equal(l_new, l_ref), n


def test_noalloc_grad_rejects_bad_arguments():
    L = esg.lib()
    P = torch.zeros(esg.MLP_PARAMS, device=DEV)
    g = torch.zeros(esg.MLP_WEIGHTS, device=DEV)
    assert L.esg_mlp_grad_noalloc(_ptr(P), None, None, 10, _ptr(g), None, None) == esg.ESG_EINVAL
    assert L.esg_mlp_grad_noalloc(_ptr(P), _ptr(P), _ptr(P), 0, _ptr(g), None, None) == \
        esg.ESG_EINVAL
