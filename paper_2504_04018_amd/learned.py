"""Training driver of the learned beam width (argument marshalling around
the library's kernels; torch holds device buffers).

Traces: for each training query, the search runs the probe (probe_hops
expansions at ef_max) and dumps the 12 features of every graph part; the
same queries are searched with fixed beams (or fixed expansion grants after
the probe) from a grid, and a query's label is log2 of the smallest beam (or
grant) whose answer reaches recall 1 against the exact answer of
esg_scan_batch (log2 of twice the grid's largest value when none does).  Every
graph part of the query is one sample with that label.  The network is
trained with esg_mlp_grad / esg_mlp_adam (mean squared error on the label),
its input normalisation taken from the training features.
"""
from __future__ import annotations

import math

import numpy as np

import paper_2504_04018_amd as esg


def exact_answers(ix, Q, l, r, k):
    """Exact top-k (float32 canonical distance) of every query: ids, dists."""
    ids, dists, _ = ix.scan(Q, l, r, k)
    return ids, dists


def per_query_recall(ids, dists, gt_dists, width, k):
    """Recall of each query: returned points whose distance does not exceed
    the k-th exact distance, over min(k, width).  Distances are the float32
    canonical distances of the returned points, so equal points compare equal."""
    import torch
    kk = torch.clamp(width, max=k)
    kth = gt_dists.gather(1, (kk - 1).clamp(min=0)[:, None])
    hit = (ids >= 0) & (dists <= kth)
    return torch.minimum(hit.sum(1), kk).float() / kk.float()


def traces(ix, Q, l, r, k, ef_grid, ef_max, probe_hops, search_kw, gt_dists, target="ef",
           label_recall=1.0):
    """Features [n_samples, 12] and labels [n_samples].

    target "ef": the label is log2 of the smallest beam of ef_grid that
    reaches recall 1.  target "hops": the beam stays ef_max and ef_grid
    lists expansion grants G after the probe; the label is log2 of the
    smallest G (a per-part hop budget of probe_hops + G) that reaches
    recall 1 (or label_recall).  Either way log2(2 * max) when none does."""
    import torch
    nq = Q.shape[0]
    feat = torch.full((nq, 2, 16), float("nan"), device=Q.device)
    ix.search_ex(Q, l, r, k, ef_max, probe_hops=probe_hops, feat_out=feat, **search_kw)
    width = r - l + 1
    grid = sorted(ef_grid)
    need = torch.full((nq,), math.log2(2 * grid[-1]), device=Q.device)
    done = torch.zeros(nq, dtype=torch.bool, device=Q.device)
    for g in grid:
        if target == "ef":
            ids, dists = ix.search_ex(Q, l, r, k, g, **search_kw)
        else:
            ids, dists = ix.search_ex(Q, l, r, k, ef_max, hop_budget=probe_hops + g, **search_kw)
        ok = per_query_recall(ids, dists, gt_dists, width, k) >= label_recall
        newly = ok & ~done
        need[newly] = math.log2(g)
        done |= ok
    torch.cuda.synchronize()
    F = feat[:, :, :12].reshape(-1, 12)
    T = need[:, None].expand(nq, 2).reshape(-1)
    keep = ~torch.isnan(F[:, 0])
    return F[keep].contiguous(), T[keep].contiguous()


def train(F, T, epochs=40, batch=8192, lr=2e-3, seed=0):
    """Adam on the mean squared error; returns the parameter tensor."""
    import torch
    dev = F.device
    g = torch.Generator(device="cpu").manual_seed(seed)
    mu = F.mean(0)
    sd = F.std(0).clamp(min=1e-3)
    w1 = torch.randn(64, 12, generator=g) * math.sqrt(2.0 / 12)
    w2 = torch.randn(64, 64, generator=g) * math.sqrt(2.0 / 64)
    w3 = torch.randn(64, generator=g) * math.sqrt(1.0 / 64)
    params = torch.cat([w1.reshape(-1), torch.zeros(64), w2.reshape(-1), torch.zeros(64), w3,
                        torch.tensor([float(T.mean())]), mu.cpu(), sd.cpu()]).float().to(dev)
    assert params.numel() == esg.MLP_PARAMS
    grad = torch.zeros(esg.MLP_WEIGHTS, device=dev)
    loss = torch.zeros(1, device=dev)
    ws = torch.zeros(esg.MLP_WORKSPACE_FLOATS, device=dev)
    m1 = torch.zeros(esg.MLP_WEIGHTS, device=dev)
    m2 = torch.zeros(esg.MLP_WEIGHTS, device=dev)
    n = F.shape[0]
    step = 0
    history = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(dev)
        tot = 0.0
        for s in range(0, n, batch):
            sel = perm[s:s + batch]
            Fb = F[sel].contiguous()
            Tb = T[sel].contiguous()
            esg.mlp_grad(params, Fb, Tb, grad, loss, ws)
            step += 1
            esg.mlp_adam(params, grad, m1, m2, step, lr)
            tot += float(loss.item()) * len(sel)
        history.append(tot / n)
    return params, history
