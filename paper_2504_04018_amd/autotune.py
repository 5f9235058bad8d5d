"""Autotuner for the batched search: times candidate launch settings on a
sample batch and keeps the fastest one whose recall meets the target.
``tune_settings`` takes the recall and the throughput of a setting from a
caller-supplied measurement (so recall can come from held-out calibration
queries while the throughput is timed on the batch itself).

Knobs: LDS visited-hash capacity (waves per CU against spills to the global
bitmap), router threshold (narrow ranges to the MFMA scan), the beam-width
calibration offset (or a fixed ef), traversal storage, and the exact scan's
rerank depth (``tune_scan``).  Every candidate runs the library's kernels;
the tuner only measures.
"""
from __future__ import annotations

import itertools
import time


def time_call(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune(ix, Q, l, r, k, ef, base_kw, recall_fn, target, grid=None, reps=3, log=None):
    """Returns (best_kw, table).  grid: dict knob -> list of values; recall_fn
    maps (ids, dists) to a mean recall."""
    grid = grid or {"hash_cap": [2048, 4096, 8192], "router_threshold": [0, 512, 1024, 2048]}
    keys = list(grid)
    table = []
    best = None
    for vals in itertools.product(*(grid[k_] for k_ in keys)):
        kw = dict(base_kw)
        kw.update(dict(zip(keys, vals)))
        out = ix.search_ex(Q, l, r, k, ef, **kw)
        rec = recall_fn(*out)
        sec = time_call(lambda: ix.search_ex(Q, l, r, k, ef, **kw), reps)
        row = dict(zip(keys, vals), recall=rec, qps=Q.shape[0] / sec)
        table.append(row)
        if log:
            log(f"tune {row}")
        if rec >= target and (best is None or row["qps"] > best[1]["qps"]):
            best = (kw, row)
    if best is None:
        best = max(((dict(base_kw, **{k_: r_[k_] for k_ in keys}), r_) for r_ in table),
                   key=lambda t: t[1]["recall"])
    return best[0], table


def tune_settings(base_kw, grid, measure, target, log=None):
    """Every combination of the grid's knobs on top of base_kw; measure(kw)
    returns (recall, qps).  Returns (best_kw, table): the fastest setting
    whose recall reaches target (else the most accurate one)."""
    keys = list(grid)
    table, best = [], None
    for vals in itertools.product(*(grid[k_] for k_ in keys)):
        kw = dict(base_kw, **dict(zip(keys, vals)))
        rec, qps = measure(kw)
        row = dict(zip(keys, vals), recall=round(rec, 5), qps=round(qps, 1))
        table.append(row)
        if log:
            log(f"tune {row}")
        if rec >= target and (best is None or qps > best[1]["qps"]):
            best = (kw, row)
    if best is None:
        best = max(((dict(base_kw, **{k_: r_[k_] for k_ in keys}), r_) for r_ in table),
                   key=lambda t: t[1]["recall"])
    return best[0], table


def tune_scan(ix, Q, l, r, k, candidates, reps=3, log=None):
    """The exact scan's rerank depth m_r: how many of a query's candidates
    (bfloat16 MFMA order) are recomputed in float32 before the certificate.
    A deeper rerank costs more per query but certifies more queries; an
    uncertified query is rescanned exactly, so every m_r gives the same
    answer and the fastest wins.  Returns (best m_r, table)."""
    table = []
    for mr in candidates:
        sec = time_call(lambda: ix.scan(Q, l, r, k, rerank_count=mr), reps)
        _, _, nfb = ix.scan(Q, l, r, k, rerank_count=mr)
        row = dict(rerank_count=mr, ms=round(sec * 1e3, 3), n_fallback=int(nfb))
        table.append(row)
        if log:
            log(f"tune scan {row}")
    best = min(table, key=lambda t: t["ms"])
    return best["rerank_count"], table
