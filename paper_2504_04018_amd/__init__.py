"""Python binding of libesg (ESG range-filtered k-NN search on MI355X).

Argument marshalling only: every step of the search runs in the HIP
kernels of ``libesg.so``; torch supplies device memory and streams.  The
library must have been built (``paper_2504_04018_amd.build.build()``); if
it is missing this module raises instead of falling back to anything else.

Names follow the C ABI in ``include/esg.h``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesg.so")

ESG_OK = 0
ESG_EINVAL = -1
ESG_ERANGE = -2
ESG_ENOMEM = -3
ESG_EIO = -4
ESG_EFORMAT = -5
ESG_EHIP = -6
ESG_EUNSUPPORTED = -7
ESG_EOVERFLOW = -8
ESG_EF_MAX = 1024
TRAV = {"f32": 0, "bf16": 1, "fp8": 2}


class EsgError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_str(status)} ({status})")
        self.status = status


METRICS = {"l2": 0, "angular": 1, "ip": 2}   # ESG_METRIC_*


class BuildParams(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("leaf", ctypes.c_int32),
                ("ef_construction", ctypes.c_int32), ("fanout", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("batch_max", ctypes.c_int32),
                ("verbose", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("metric", ctypes.c_int32)]


class IndexInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("leaf", ctypes.c_int32), ("fanout", ctypes.c_int32),
                ("n_depth", ctypes.c_int32), ("c_den", ctypes.c_int32),
                ("has_bf16", ctypes.c_int32), ("has_fp8", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("metric", ctypes.c_int32),
                ("dq", ctypes.c_int32), ("max_norm2", ctypes.c_double)]


class PartTrace(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("depth", ctypes.c_int32), ("heap", ctypes.c_int64),
                ("a", ctypes.c_int64), ("b", ctypes.c_int64), ("x", ctypes.c_int64),
                ("y", ctypes.c_int64), ("hops", ctypes.c_int64), ("n_visited", ctypes.c_int64),
                ("ticks", ctypes.c_int64)]


TRACE_FIELDS = [f[0] for f in PartTrace._fields_]
TRACE_INT64S = ctypes.sizeof(PartTrace) // 8


class SearchOpts(ctypes.Structure):
    _fields_ = [("traversal", ctypes.c_int32), ("rerank", ctypes.c_int32),
                ("cand_cap", ctypes.c_int32), ("hash_cap", ctypes.c_int32),
                ("hop_budget", ctypes.c_int64), ("router_threshold", ctypes.c_int64),
                ("use_graph", ctypes.c_int32), ("scan_rerank", ctypes.c_int32),
                ("mlp", ctypes.c_void_p), ("probe_hops", ctypes.c_int32),
                ("mlp_delta", ctypes.c_float), ("mlp_target", ctypes.c_int32),
                ("feat_out", ctypes.c_void_p),
                ("trace", ctypes.c_void_p),
                ("visited", ctypes.c_void_p), ("visited_cap", ctypes.c_int64),
                ("n_invalid", ctypes.c_void_p), ("part_ef", ctypes.c_void_p)]


class ScanOpts(ctypes.Structure):
    _fields_ = [("rerank_count", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("certified", ctypes.c_void_p), ("n_fallback", ctypes.c_void_p)]


_lib = None

# Every symbol include/esg.h declares, with (restype, argtypes).
_I32, _I64, _VP, _CP = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_char_p
SIGNATURES = {
    "esg_build_index": (_I32, [_VP, _VP, _I64, _I32, _VP, _CP]),
    "esg_build_index_gpu": (_I32, [_VP, _VP, _I64, _I32, _VP, _I32, _CP]),
    "esg_load_index": (_I32, [_CP, _I32, _VP]),
    "esg_index_add_storage": (_I32, [_VP, _I32, _VP]),
    "esg_index_info": (_I32, [_VP, _VP]),
    "esg_index_copy_storage": (_I32, [_VP, _I32, _VP, _I64]),
    "esg_free_index": (None, [_VP]),
    "esg_status_str": (_CP, [_I32]),
    "esg_search_batch": (_I32, [_VP, _VP, _VP, _VP, _I64, _I32, _I32, _VP, _VP, _VP]),
    "esg_search_batch_ex": (_I32, [_VP, _VP, _VP, _VP, _VP, _I64, _I32, _I32, _VP, _VP, _VP]),
    "esg_index_reserve": (_I32, [_VP, _I64, _I64]),
    "esg_scan_batch": (_I32, [_VP, _VP, _VP, _VP, _VP, _I64, _I32, _VP, _VP, _VP]),
    "esg_mlp_forward": (_I32, [_VP, _VP, _I64, _VP, _VP]),
    "esg_mlp_grad": (_I32, [_VP, _VP, _VP, _I64, _VP, _VP, _VP, _VP]),
    "esg_mlp_adam": (_I32, [_VP, _VP, _VP, _VP, _I64, ctypes.c_float, _VP]),
    "esg_mlp_grad_noalloc": (_I32, [_VP, _VP, _VP, _I64, _VP, _VP, _VP]),
}
MLP_FEATURES, MLP_WEIGHTS, MLP_PARAMS = 12, 5057, 5081
MLP_WORKSPACE_FLOATS = 512 * 5058


def lib() -> ctypes.CDLL:
    """Loads libesg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2504_04018_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_str(status: int) -> str:
    return lib().esg_status_str(status).decode()


def _check(status: int, what: str):
    if status != ESG_OK:
        raise EsgError(status, what)


def build_index(X: np.ndarray, attr: np.ndarray, path: str, degree: int = 16, leaf: int = 1024,
                ef_construction: int = 200, threads: int = 0, batch_max: int = 0,
                verbose: bool = False, fanout: int = 2, layout: str = "tree",
                metric: str = "l2", device: int | None = None) -> None:
    """esg_build_index (host threads) or, with a HIP `device`,
    esg_build_index_gpu (insertion rounds on that device; the same file
    byte for byte): the index file -- layout "tree": the
    HBI-2D segment tree (Alg. 3) of the given fanout (elastic constant
    1/fanout); layout "chain": the half-bounded HBI-1D index (Alg. 2),
    prefix and suffix graphs of sizes N, ceil(N/B), ... with B = fanout.
    metric "l2", "angular" (rows stored at unit norm) or "ip" (maximum inner
    product: rows stored as [x, sqrt(M^2 - |x|^2)], queries stay [n, d])."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    attr = np.ascontiguousarray(attr, dtype=np.float64)
    if X.ndim != 2 or attr.shape != (X.shape[0],):
        raise ValueError("X must be [n,d] and attr [n]")
    p = BuildParams(degree, leaf, ef_construction, fanout, threads, batch_max, int(verbose),
                    {"tree": 0, "chain": 1}[layout], METRICS[metric])
    if device is None:
        st = lib().esg_build_index(X.ctypes.data, attr.ctypes.data, X.shape[0], X.shape[1],
                                   ctypes.byref(p), path.encode())
        _check(st, "esg_build_index")
    else:
        st = lib().esg_build_index_gpu(X.ctypes.data, attr.ctypes.data, X.shape[0], X.shape[1],
                                       ctypes.byref(p), int(device), path.encode())
        _check(st, "esg_build_index_gpu")


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Index:
    """A loaded index (esg_load_index); owns its device memory until free()."""

    def __init__(self, path: str, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().esg_load_index(path.encode(), device, ctypes.byref(h)), "esg_load_index")
        self._h = h
        self.device = device
        self.path = path
        inf = self.info()
        self.n, self.d = inf["n"], inf["d"]
        self.dq = inf["dq"]             # values per query row
        self.metric = {v: k for k, v in METRICS.items()}[inf["metric"]]
        self.max_norm2 = inf["max_norm2"]

    def info(self) -> dict:
        out = IndexInfo()
        _check(lib().esg_index_info(self._h, ctypes.byref(out)), "esg_index_info")
        return {f[0]: getattr(out, f[0]) for f in IndexInfo._fields_}

    def add_storage(self, kind: str, stream=None) -> None:
        _check(lib().esg_index_add_storage(self._h, TRAV[kind], _stream_ptr(stream)),
               "esg_index_add_storage")

    def copy_storage(self, kind: str):
        """Host copy of a device vector store: float32 [n,d], bfloat16 bits
        [n,d] (uint16), or (fp8 codes [n,d] uint8, scales [n] float32)."""
        n, d = self.n, self.d
        if kind == "f32":
            out = np.empty((n, d), np.float32)
        elif kind == "bf16":
            out = np.empty((n, d), np.uint16)
        else:
            out = np.empty(n * d + 4 * n, np.uint8)
        _check(lib().esg_index_copy_storage(self._h, TRAV[kind], out.ctypes.data, out.nbytes),
               "esg_index_copy_storage")
        if kind == "fp8":
            return out[:n * d].reshape(n, d), out[n * d:].view(np.float32)
        return out

    def reserve(self, max_queries: int, max_windows: int) -> None:
        """esg_index_reserve: workspace of the brute-force scan and the router."""
        _check(lib().esg_index_reserve(self._h, max_queries, max_windows), "esg_index_reserve")

    def scan(self, queries, l, r, k: int, ids=None, dists=None, rerank_count: int = 0,
             certified=None, exact: bool = False, stream=None):
        """esg_scan_batch: exact range-filtered k-NN; returns (ids, dists, n_fallback)."""
        import torch
        nq = queries.shape[0]
        dev = queries.device
        qp = _dev(queries, torch.float32, (nq, self.dq), "queries")
        lp = _dev(l, torch.int64, (nq,), "l")
        rp = _dev(r, torch.int64, (nq,), "r")
        if ids is None:
            ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
        if dists is None:
            dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
        nfb = ctypes.c_int64(0)
        o = ScanOpts(rerank_count, 1 if exact else 0,
                     None if certified is None else certified.data_ptr(), ctypes.addressof(nfb))
        st = lib().esg_scan_batch(self._h, ctypes.byref(o), qp, lp, rp, nq, k,
                                  _dev(ids, torch.int64, (nq, k), "ids"),
                                  _dev(dists, torch.float32, (nq, k), "dists"),
                                  _stream_ptr(stream))
        _check(st, "esg_scan_batch")
        return ids, dists, nfb.value

    def search(self, queries, l, r, k: int, ef: int, ids=None, dists=None, stream=None):
        """esg_search_batch on device tensors; returns (ids int64 [nq,k], dists f32 [nq,k])."""
        return self.search_ex(queries, l, r, k, ef, ids=ids, dists=dists, stream=stream,
                              opts=None)

    def search_ex(self, queries, l, r, k: int, ef: int, traversal: str = "f32",
                  rerank: bool = False, cand_cap: int = 0, hash_cap: int = 0,
                  hop_budget: int = -1, router_threshold: int = 0, use_graph: bool = False,
                  scan_rerank: int = 0, mlp=None, probe_hops: int = 0, mlp_delta: float = 0.0,
                  mlp_target: int = 0, feat_out=None, trace=None, visited=None, visited_cap: int = 0,
                  n_invalid=None, part_ef=None, ids=None, dists=None, stream=None, opts="build"):
        import torch
        nq = queries.shape[0]
        dev = queries.device
        qp = _dev(queries, torch.float32, (nq, self.dq), "queries")
        lp = _dev(l, torch.int64, (nq,), "l")
        rp = _dev(r, torch.int64, (nq,), "r")
        if ids is None:
            ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
        if dists is None:
            dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
        ip = _dev(ids, torch.int64, (nq, k), "ids")
        dp = _dev(dists, torch.float32, (nq, k), "dists")
        if opts is None:
            st = lib().esg_search_batch(self._h, qp, lp, rp, nq, k, ef, ip, dp,
                                        _stream_ptr(stream))
        else:
            o = SearchOpts(TRAV[traversal], int(rerank), cand_cap, hash_cap, hop_budget,
                           router_threshold, int(use_graph), scan_rerank,
                           None if mlp is None else mlp.data_ptr(), probe_hops, mlp_delta,
                           mlp_target,
                           None if feat_out is None else feat_out.data_ptr(),
                           None if trace is None else trace.data_ptr(),
                           None if visited is None else visited.data_ptr(),
                           visited_cap, None if n_invalid is None else n_invalid.data_ptr(),
                           None if part_ef is None else
                           _dev(part_ef, torch.int32, (nq, 2), "part_ef"))
            st = lib().esg_search_batch_ex(self._h, ctypes.byref(o), qp, lp, rp, nq, k, ef, ip, dp,
                                           _stream_ptr(stream))
        _check(st, "esg_search_batch")
        return ids, dists

    def free(self) -> None:
        if getattr(self, "_h", None):
            lib().esg_free_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def trace_tensor(nq: int, device):
    """Device buffer for per-part trace records ([nq, 2] esg_part_trace)."""
    import torch
    return torch.zeros((nq, 2, TRACE_INT64S), dtype=torch.int64, device=device)


def decode_trace(t) -> dict:
    """Host view of a trace tensor: dict of [nq,2] numpy arrays."""
    a = t.cpu().numpy()
    kd = a[..., 0].copy().view(np.int32).reshape(a.shape[0], a.shape[1], 2)
    out = {"kind": kd[..., 0].astype(np.int64), "depth": kd[..., 1].astype(np.int64)}
    for i, name in enumerate(["heap", "a", "b", "x", "y", "hops", "n_visited", "ticks"]):
        out[name] = a[..., 1 + i]
    return out


def mlp_forward(params, feats, out=None, stream=None):
    """esg_mlp_forward on device tensors (float32 [5081], [n,12]) -> [n]."""
    import torch
    n = feats.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=feats.device)
    _check(lib().esg_mlp_forward(_dev(params, torch.float32, (MLP_PARAMS,), "params"),
                                 _dev(feats, torch.float32, (n, MLP_FEATURES), "feats"), n,
                                 _dev(out, torch.float32, (n,), "out"), _stream_ptr(stream)),
           "esg_mlp_forward")
    return out


def mlp_grad(params, feats, target, grad, loss, workspace, stream=None):
    """esg_mlp_grad: grad[5057] and loss[1] of the mean squared error."""
    import torch
    n = feats.shape[0]
    _check(lib().esg_mlp_grad(_dev(params, torch.float32, (MLP_PARAMS,), "params"),
                              _dev(feats, torch.float32, (n, MLP_FEATURES), "feats"),
                              _dev(target, torch.float32, (n,), "target"), n,
                              _dev(grad, torch.float32, (MLP_WEIGHTS,), "grad"),
                              _dev(loss, torch.float32, (1,), "loss"),
                              _dev(workspace, torch.float32, (MLP_WORKSPACE_FLOATS,), "workspace"),
                              _stream_ptr(stream)), "esg_mlp_grad")


def mlp_grad_noalloc(params, feats, target, grad, loss, stream=None):
    """esg_mlp_grad_noalloc: as mlp_grad, with the library's own scratch
    (allocates nothing; calls on one GPU must not overlap)."""
    import torch
    n = feats.shape[0]
    _check(lib().esg_mlp_grad_noalloc(_dev(params, torch.float32, (MLP_PARAMS,), "params"),
                                      _dev(feats, torch.float32, (n, MLP_FEATURES), "feats"),
                                      _dev(target, torch.float32, (n,), "target"), n,
                                      _dev(grad, torch.float32, (MLP_WEIGHTS,), "grad"),
                                      _dev(loss, torch.float32, (1,), "loss"),
                                      _stream_ptr(stream)), "esg_mlp_grad_noalloc")


def mlp_adam(params, grad, m1, m2, step, lr, stream=None):
    import torch
    _check(lib().esg_mlp_adam(_dev(params, torch.float32, (MLP_PARAMS,), "params"),
                              _dev(grad, torch.float32, (MLP_WEIGHTS,), "grad"),
                              _dev(m1, torch.float32, (MLP_WEIGHTS,), "m1"),
                              _dev(m2, torch.float32, (MLP_WEIGHTS,), "m2"), step, lr,
                              _stream_ptr(stream)), "esg_mlp_adam")
