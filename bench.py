#!/usr/bin/env python3
"""Benchmark: QPS at recall@10 >= 0.95 for ESG range-filtered search on one MI355X.

Workload (default): SIFT-shaped, N = 1,000,000 uint8-valued vectors in
d = 128 (64-centre clipped, rounded mixture), attribute = random
permutation, 10,000 queries in 11 equal buckets of range width
floor(N * 2^-b), k = 10.  The synthetic set stands in for SIFT1M.

A step is one batch search of all queries (selector, beam search / leaf
scan, merge, top-k) with the inputs resident in HBM.  The bench sweeps ef
for float32 traversal and for bfloat16 traversal with the float32 rerank,
keeps the operating point with the highest QPS whose mean recall@10
(tie-aware, against exact ground truth) is >= 0.95, and times K steps of
it.  One JSON line is printed.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
EF_GRID = [16, 24, 32, 48, 64, 96, 128, 192, 256]
TARGET_RECALL = 0.95


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="shrink N (default: full 1M)")
    ap.add_argument("--nq", type=int, default=None, help="shrink the query count")
    ap.add_argument("--cache-dir", default=os.environ.get("ESG_BENCH_CACHE", "/tmp/esg_bench"))
    ap.add_argument("--cpu-sample", type=int, default=2000,
                    help="queries timed on the CPU oracle (bounded sample)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--modes", default="f32,bf16")
    ap.add_argument("--mode", default=None, help="fixed operating point: skip the sweep")
    ap.add_argument("--ef", type=int, default=None, help="fixed operating point: skip the sweep")
    return ap.parse_args()


def ground_truth_kth(X_pos, Q, l, r, k, dev):
    """k-th smallest exact squared distance inside each query's range
    (measurement only: it judges recall).  Integer-valued data keeps every
    float32 partial sum exact (< 2^24), so the GEMM form is exact here."""
    import torch
    torch.backends.cuda.matmul.allow_tf32 = False
    Xt = torch.from_numpy(X_pos).to(dev)
    xn = (Xt * Xt).sum(1)
    Qt = torch.from_numpy(Q).to(dev)
    qn = (Qt * Qt).sum(1)
    lt = torch.from_numpy(l).to(dev)
    rt = torch.from_numpy(r).to(dev)
    nq = Q.shape[0]
    n = X_pos.shape[0]
    best = torch.full((nq, k), float("inf"), device=dev)
    chunk, qb = 65536, 2048
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        pos = torch.arange(s, e, device=dev)
        for q0 in range(0, nq, qb):
            q1 = min(nq, q0 + qb)
            hit = (lt[q0:q1] <= e - 1) & (rt[q0:q1] >= s)
            if not bool(hit.any()):
                continue
            D = xn[s:e][None, :] + qn[q0:q1, None] - 2.0 * (Qt[q0:q1] @ Xt[s:e].T)
            mask = (pos[None, :] < lt[q0:q1, None]) | (pos[None, :] > rt[q0:q1, None])
            D = D.masked_fill(mask, float("inf"))
            kk = min(k, e - s)
            cand = torch.topk(D, kk, dim=1, largest=False).values
            best[q0:q1] = torch.topk(torch.cat([best[q0:q1], cand], 1), k, dim=1,
                                     largest=False).values
    width = torch.from_numpy(r - l + 1).to(dev)
    kk = torch.clamp(width, max=k) - 1
    return best.gather(1, kk[:, None])[:, 0].cpu().numpy().astype(np.float64)


def recall_at_k(ids, pos_of, X_pos, Q, l, r, dk, k):
    """Mean tie-aware recall: returned in-range points whose exact distance
    is <= the k-th true one, over min(k, width)."""
    pos = np.where(ids >= 0, pos_of[np.maximum(ids, 0)], -1)
    ok = (pos >= l[:, None]) & (pos <= r[:, None]) & (ids >= 0)
    safe = np.where(ok, pos, 0)
    diff = X_pos[safe].astype(np.float64) - Q[:, None, :].astype(np.float64)
    d = np.sum(diff * diff, axis=2)
    hit = ok & (d <= dk[:, None])
    kk = np.minimum(k, r - l + 1)
    return float(np.mean(np.minimum(hit.sum(1), kk) / kk))


def algorithmic_bytes(trace, d, R, k, ef, elem_bytes, rerank):
    """Bytes the method itself must move for one batch: per graph part
    |V|*d*s (vectors) + hops*R*4 (adjacency rows) + d*4 (query); per leaf
    scan w*d*4 + d*4; the float32 rerank adds min(ef, |V|)*d*4 per graph
    part; outputs k*12 per query."""
    kind, nv, hops = trace["kind"], trace["n_visited"], trace["hops"]
    g = kind == 1
    s = kind == 2
    b = (nv[g] * d * elem_bytes).sum() + (hops[g] * R * 4).sum() + g.sum() * d * 4
    b += (nv[s] * d * 4).sum() + s.sum() * d * 4
    if rerank:
        b += (np.minimum(ef, nv[g]) * d * 4).sum()
    b += kind.shape[0] * k * 12
    return float(b)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_2504_04018_amd as esg
    import synth

    dev = torch.device("cuda:0")
    t0 = time.time()
    w = synth.make_workload(1, n=args.n, nq=args.nq)
    n, d, k = w["n"], w["d"], w["k"]
    nq = len(w["Q"])
    log(f"workload {w['name']} n={n} d={d} nq={nq} generated in {time.time() - t0:.1f}s")
    os.makedirs(args.cache_dir, exist_ok=True)
    tag = synth.sha256_of(w["X"][:1000], w["attr"][:1000])[:12]
    path = os.path.join(args.cache_dir, f"sift_{n}_R{w['degree']}_{tag}.esgi")
    if not os.path.exists(path):
        t0 = time.time()
        esg.build_index(w["X"], w["attr"].astype(np.float64), path + ".tmp", degree=w["degree"],
                        leaf=w["leaf"], ef_construction=w["ef_construction"], verbose=True)
        os.replace(path + ".tmp", path)
        log(f"index built in {time.time() - t0:.1f}s")
    ix = esg.Index(path, 0)
    ix.add_storage("bf16")
    info = ix.info()
    # position order (attribute ranks) of the vectors, from the generator
    order = np.argsort(w["attr"], kind="stable")
    X_pos = np.ascontiguousarray(w["X"][order])
    pos_of = np.empty(n, np.int64)
    pos_of[order] = np.arange(n)

    Q, l, r = w["Q"], w["l"], w["r"]
    Qd = torch.from_numpy(Q).to(dev)
    ld = torch.from_numpy(l).to(dev)
    rd = torch.from_numpy(r).to(dev)
    t0 = time.time()
    dk = ground_truth_kth(X_pos, Q, l, r, k, dev)
    log(f"ground truth in {time.time() - t0:.1f}s")

    modes = {"f32": dict(traversal="f32", rerank=False, elem=4),
             "bf16": dict(traversal="bf16", rerank=True, elem=2)}
    ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
    dists = torch.empty((nq, k), dtype=torch.float32, device=dev)

    def run(mode, ef, trace=None):
        m = modes[mode]
        ix.search_ex(Qd, ld, rd, k, ef, traversal=m["traversal"], rerank=m["rerank"],
                     trace=trace, ids=ids, dists=dists)

    def time_it(mode, ef, reps):
        torch.cuda.synchronize()
        s = time.perf_counter()
        for _ in range(reps):
            run(mode, ef)
        torch.cuda.synchronize()
        return (time.perf_counter() - s) / reps

    sweep = []
    fixed = args.mode is not None and args.ef is not None
    for mode in ([args.mode] if fixed else args.modes.split(",")):
        for ef in ([args.ef] if fixed else EF_GRID):
            if ef < k:
                continue
            run(mode, ef)
            torch.cuda.synchronize()
            rec = recall_at_k(ids.cpu().numpy(), pos_of, X_pos, Q, l, r, dk, k)
            sec = time_it(mode, ef, 1 if fixed else 3)
            sweep.append(dict(mode=mode, ef=ef, recall=round(rec, 5), qps=round(nq / sec, 1)))
            log(f"sweep {mode} ef={ef} recall={rec:.4f} qps={nq / sec:,.0f}")
            if rec >= 0.995:
                break
    ok = [s for s in sweep if s["recall"] >= TARGET_RECALL]
    if not ok:
        best = max(sweep, key=lambda s: s["recall"])
    else:
        best = max(ok, key=lambda s: s["qps"])
    plain = [s for s in ok if s["mode"] == "f32"]
    plain_best = max(plain, key=lambda s: s["qps"]) if plain else None
    mode, ef = best["mode"], best["ef"]
    log(f"operating point: {mode} ef={ef} recall={best['recall']}")

    # algorithmic bytes of one step, from a traced (identical) run
    tr = esg.trace_tensor(nq, dev)
    run(mode, ef, trace=tr)
    torch.cuda.synchronize()
    trace = esg.decode_trace(tr)
    alg_bytes = algorithmic_bytes(trace, d, info["degree"], k, ef, modes[mode]["elem"],
                                  modes[mode]["rerank"])

    # timed region
    for _ in range(args.warmup):
        run(mode, ef)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record()
        run(mode, ef)
        ends[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
    ms_per_step = wall * 1000.0 / args.steps
    qps = nq / (ms_per_step / 1000.0)
    achieved = alg_bytes / (kern_ms / 1000.0) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.time()
        oix = oracle.read_index(path)
        if mode == "bf16":
            oix.with_bf16()
        S = min(args.cpu_sample, nq)
        sel = np.arange(S)
        kind = oracle.DIST_BF16 if mode == "bf16" else oracle.DIST_F32
        s = time.perf_counter()
        oracle.query_batch(oix, Q[sel], l[sel], r[sel], k, ef, ef, -1, kind,
                           int(modes[mode]["rerank"]))
        el = time.perf_counter() - s
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": round(S / el, 1), "unit": "queries/s", "cores": cores, "kind": "oracle",
               "sample": f"first {S} of the {nq} queries, same ef={ef} and traversal ({mode}), "
                         f"OpenMP over queries; {el:.1f}s"}
        log(f"cpu oracle {S / el:,.0f} q/s on {cores} cores ({time.time() - t0:.1f}s incl. load)")

    out = {
        "metric": "QPS at recall@10>=0.95 (1 MI355X), with achieved HBM GB/s",
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f32" if mode == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": f"sift-shaped N={n} d={d} uint8-valued, {nq} queries, 11 range "
                               f"buckets 2^-b*N, k={k}", "mode": mode, "ef": ef,
                   "recall_at_10": best["recall"], "leaf": info["leaf"],
                   "degree": info["degree"], "n_depth": info["n_depth"]},
        "plain_f32": plain_best,
        "sweep": sweep,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "search_kernel", "kernel_ms": round(kern_ms, 4),
                     "alg_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ix.free()


if __name__ == "__main__":
    main()
