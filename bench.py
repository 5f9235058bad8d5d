#!/usr/bin/env python3
"""Benchmark: QPS at recall@10 >= 0.95 on one MI355X, learned + batched +
bfloat16 search against the plain float32 fixed-ef search.

Default workload (--workload deep): DEEP-shaped batched mixed ranges,
N = 1,000,000 unit-norm vectors in d = 96 (256-centre mixture), attribute =
random permutation, 100,000 queries with range widths log-uniform over
[10, N], k = 10.  The synthetic set stands in for DEEP1M.  --workload sift
runs the SIFT-shaped set (1M x 128 uint8-valued, 10,000 queries in 11
width buckets).

A step is one batch search of all queries with the inputs resident in HBM.
Three forms are measured, each at its fastest setting whose mean recall@10
against exact ground truth (the library's brute-force scan) is >= 0.95:
  plain_f32          float32 traversal, one fixed ef for every query;
  fixed_batched      traversal (bfloat16 + float32 rerank, or float32), router
                     threshold (narrow ranges to the MFMA scan) and
                     visited-hash size picked by the autotuner, one replayed
                     hipGraph, fixed ef;
  learned_batched    the same with the per-part beam width (or stopping
                     step) predicted by the network trained here on traces
                     of 200,000 separate training queries (GPU kernels).
Settings are swept on the evaluation queries for every form alike (a
QPS/recall frontier).  K steps of the learned form are timed and give
`value`; the other two are reported beside it.  One JSON line is printed.
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
MFMA_BF16_PEAK_TFLOPS = 2500.0
TARGET_RECALL = 0.95
EF_GRID = [10, 12, 14, 16, 18, 20, 22, 24, 28, 32, 40, 48, 64, 96, 100, 112, 128, 192, 256, 384, 512, 768, 1024]
DELTA_GRID = [-1.0, -0.75, -0.5, -0.375, -0.25, -0.125, 0.0, 0.25, 0.5]
LABEL_EF_GRID = [10, 12, 14, 16, 18, 20, 22, 24, 28, 32, 40, 48, 64, 96, 128, 192, 256]
LABEL_HOP_GRID = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="deep", choices=["deep", "sift", "embedding"],
                    help="embedding: unit-norm d=768, k=100, fp8 storage (N defaults to 200,000)")
    ap.add_argument("--n", type=int, default=None, help="shrink N (default: the full workload)")
    ap.add_argument("--nq", type=int, default=None, help="shrink the query count")
    ap.add_argument("--ntrain", type=int, default=200_000, help="training traces")
    ap.add_argument("--ef-max", type=int, default=32, help="beam of the learned form")
    ap.add_argument("--probe-hops", type=int, default=4)
    ap.add_argument("--reps", type=int, default=5, help="timed repetitions per sweep point")
    ap.add_argument("--cache-dir", default=os.environ.get("ESG_BENCH_CACHE", "/tmp/esg_bench"))
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU oracle baseline: chunks of queries until this much time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-only", action="store_true", help="skip the learned variant")
    ap.add_argument("--fixed-ef", type=int, default=None, help="fixed-ef forms at this ef only")
    ap.add_argument("--traversal", choices=["f32", "bf16"], default=None,
                    help="batched forms: this traversal only (default: autotuned)")
    ap.add_argument("--router", type=int, default=None, help="router threshold (default: tuned)")
    ap.add_argument("--hash-cap", type=int, default=None, help="visited hash (default: tuned)")
    ap.add_argument("--target", choices=["ef", "hops"], default=None,
                    help="learned target (default: both, the faster kept)")
    ap.add_argument("--delta", type=float, default=None, help="learned offset (default: swept)")
    ap.add_argument("--scan-only", action="store_true",
                    help="time only the exact MFMA range scan over the workload's queries "
                         "(MFMA roofline), print one JSON line and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES of device memory 5 times and exit (calibrates the "
                         "HBM byte counters against a transfer of known size)")
    return ap.parse_args()


def algorithmic_bytes(trace, d, R, k, m, elem_bytes, rerank):
    """Bytes the method itself must move: per graph part |V|*d*s (vectors)
    + hops*R*4 (adjacency rows) + d*4 (query); per leaf scan w*d*4 + d*4;
    the float32 rerank of the final Q adds min(m, |V|, width)*d*4 per graph
    part (m: the part's beam, per part when the network chose it); outputs
    k*12 per query."""
    kind, nv, hops = trace["kind"], trace["n_visited"], trace["hops"]
    g = kind == 1
    s = kind == 2
    b = (nv[g] * d * elem_bytes).sum() + (hops[g] * R * 4).sum() + g.sum() * d * 4
    b += (nv[s] * d * 4).sum() + s.sum() * d * 4
    if rerank:
        w = trace["y"] - trace["x"] + 1
        b += (np.minimum(np.minimum(m, nv), w)[g] * d * 4).sum()
    b += kind.shape[0] * k * 12
    return float(b)


def kernel_sources_sha256():
    """Hash of the library's kernel sources: a stored traffic figure is used
    only while these are unchanged."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2504_04018_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".h", ".hip")):
            h.update(f.encode())
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def stored_traffic(key):
    """HBM bytes per launch from the committed rocprofv3 counter summaries
    (FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size), for the
    same operating point and unchanged kernel sources; else None."""
    pdir = os.path.join(ROOT, "profiles")
    sha = kernel_sources_sha256()
    for f in sorted(os.listdir(pdir)) if os.path.isdir(pdir) else []:
        for line in open(os.path.join(pdir, f)):
            if line.startswith("traffic-record: "):
                rec = json.loads(line[len("traffic-record: "):])
                if rec.get("sources_sha256") == sha and rec.get("key") == key:
                    return rec["hbm_bytes_per_launch"]
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    if args.copy_probe:
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4, "copies": 5}))
        return

    import paper_2504_04018_amd as esg
    from paper_2504_04018_amd import autotune, learned
    import synth

    dev = torch.device("cuda:0")
    cid = {"deep": 2, "sift": 1, "embedding": 3}[args.workload]
    if cid == 3 and args.n is None:
        args.n = 200_000
    t0 = time.time()
    w = synth.make_workload(cid, n=args.n, nq=args.nq)
    n, d, k = w["n"], w["d"], w["k"]
    nq = len(w["Q"])
    log(f"workload {w['name']} n={n} d={d} nq={nq} generated in {time.time() - t0:.1f}s")
    os.makedirs(args.cache_dir, exist_ok=True)
    tag = synth.sha256_of(w["X"][:1000], w["attr"][:1000])[:12]
    path = os.path.join(args.cache_dir, f"{args.workload}_{n}_R{w['degree']}_{tag}.esgi")
    if not os.path.exists(path):
        t0 = time.time()
        esg.build_index(w["X"], w["attr"].astype(np.float64), path + ".tmp", degree=w["degree"],
                        leaf=w["leaf"], ef_construction=w["ef_construction"], verbose=True)
        os.replace(path + ".tmp", path)
        log(f"index built in {time.time() - t0:.1f}s")
    X = w.pop("X")                        # kept for the float64 distance check
    ix = esg.Index(path, 0)
    ix.add_storage("bf16")
    if cid == 3:
        ix.add_storage("fp8")
    ix.reserve(max(nq, args.ntrain), 262144)
    info = ix.info()

    def dev_t(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    Q, l, r = dev_t(w["Q"]), dev_t(w["l"]), dev_t(w["r"])
    width = r - l + 1
    t0 = time.time()
    gt_ids, gt_d = learned.exact_answers(ix, Q, l, r, k)
    torch.cuda.synchronize()
    log(f"exact ground truth (MFMA scan) in {time.time() - t0:.1f}s")

    if args.scan_only:
        # exact scan: algorithmic flops 2*w*d per query (in-range points only)
        wsum = float((width).sum().item())
        alg_flops = 2.0 * wsum * d
        t_ms, nfb = [], 0
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, nfb = ix.scan(Q, l, r, k)
            torch.cuda.synchronize()
            if i >= args.warmup:
                t_ms.append((time.perf_counter() - t0) * 1000.0)
        ms = float(np.median(t_ms))
        tf = alg_flops / (ms / 1000.0) / 1e12
        print(json.dumps({"scan_only": True, "workload": args.workload, "n": n, "d": d, "nq": nq,
                          "k": k, "ms_per_batch": round(ms, 3), "queries_per_s": round(nq / ms * 1e3),
                          "alg_tflop_per_batch": round(alg_flops / 1e12, 3),
                          "alg_tflops": round(tf, 1), "bf16_peak_tflops": MFMA_BF16_PEAK_TFLOPS,
                          "frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 4), "n_fallback": int(nfb)}))
        return

    def recall(ids, dists):
        return float(learned.per_query_recall(ids, dists, gt_d, width, k).mean().item())

    ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
    dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
    sweep = []

    def point(variant, ef, kw, **extra):
        ix.search_ex(Q, l, r, k, ef, ids=ids, dists=dists, **kw)
        rec = recall(ids, dists)
        sec = autotune.time_call(lambda: ix.search_ex(Q, l, r, k, ef, ids=ids, dists=dists, **kw),
                                 args.reps)
        row = dict(variant=variant, ef=ef, traversal=kw.get("traversal", "f32"),
                   recall=round(rec, 5), qps=round(nq / sec, 1), **extra)
        sweep.append(row)
        log(f"{variant} ef={ef} {extra} recall={rec:.4f} qps={nq / sec:,.0f}")
        return row

    def best_of(rows):
        ok = [s for s in rows if s["recall"] >= TARGET_RECALL]
        return max(ok, key=lambda s: s["qps"]) if ok else None

    def fixed_sweep(variant, kw):
        rows, hits = [], 0
        for ef in ([args.fixed_ef] if args.fixed_ef else EF_GRID):
            if ef < k:
                continue
            rows.append(point(variant, ef, kw))
            hits += rows[-1]["recall"] >= TARGET_RECALL
            if hits >= 3:                      # QPS only falls from here on
                break
        return best_of(rows) or max(rows, key=lambda s: s["recall"])

    # ---- plain: float32 traversal, fixed ef -------------------------------------
    plain_kw = dict(traversal="f32")
    plain_best = fixed_sweep("plain_f32", plain_kw)

    # ---- batched + bfloat16, fixed ef, autotuned launch settings --------------------
    fixed_best = learned_best = train_info = None
    lkw = None
    if not args.plain_only:
        base = dict(rerank=True, use_graph=True)
        tuned, _ = autotune.tune(
            ix, Q, l, r, k, plain_best["ef"], base, recall, 0.0,
            grid={"traversal": [args.traversal] if args.traversal else
                  (["fp8", "bf16", "f32"] if cid == 3 else ["bf16", "f32"]),
                  "router_threshold": [args.router] if args.router is not None else [0, 512, 2048],
                  "hash_cap": [args.hash_cap] if args.hash_cap else [4096, 8192]},
            reps=args.reps, log=log)
        tuned["rerank"] = tuned["traversal"] != "f32"
        bkw = {kk: tuned[kk] for kk in ("traversal", "rerank", "use_graph", "router_threshold",
                                         "hash_cap")}
        fixed_best = fixed_sweep("fixed_batched", bkw)

    if not args.plain_only and args.ef_max < k:
        log(f"learned form skipped: --ef-max {args.ef_max} < k = {k}")
    elif not args.plain_only:
        # ---- learned: traces of separate training queries, GPU training ------------------
        t0 = time.time()
        wt = synth.make_workload(cid, n=n, nq=args.ntrain, query_stream=5000, range_stream=6000)
        del wt["X"]
        Qt, lt, rt = dev_t(wt["Q"]), dev_t(wt["l"]), dev_t(wt["r"])
        _, gt_dt = learned.exact_answers(ix, Qt, lt, rt, k)
        tkw = {kk: v for kk, v in bkw.items() if kk != "use_graph"}
        train_info = {}
        cands = []
        for target, grid in (("ef", LABEL_EF_GRID), ("hops", LABEL_HOP_GRID)):
            if args.target and target != args.target:
                continue
            t1 = time.time()
            g = [v for v in grid if target == "hops" or v <= args.ef_max]
            F, T = learned.traces(ix, Qt, lt, rt, k, g, args.ef_max, args.probe_hops, tkw, gt_dt,
                                  target=target)
            params, hist = learned.train(F, T)
            train_info[target] = dict(traces=int(F.shape[0]), queries=args.ntrain,
                                      first_mse=round(hist[0], 4), final_mse=round(hist[-1], 4),
                                      seconds=round(time.time() - t1, 2))
            log(f"learned target={target}: {F.shape[0]} part traces, mse {hist[0]:.3f} -> "
                f"{hist[-1]:.3f} in {time.time() - t1:.1f}s")
            cands.append((target, params))
            del F, T
        del Qt, lt, rt, gt_dt
        # the network is evaluated with the tuned traversal and with the other one
        travs = [bkw["traversal"]] + ([] if args.traversal else
                                      [t for t in ("bf16", "f32") if t != bkw["traversal"]])
        rows = []
        for target, params in cands:
            for trav in travs:
                kw = dict(bkw, traversal=trav, rerank=trav != "f32", mlp=params,
                          probe_hops=args.probe_hops, mlp_target=1 if target == "hops" else 0)
                for delta in ([args.delta] if args.delta is not None else DELTA_GRID):
                    rows.append(point("learned_batched", args.ef_max, dict(kw, mlp_delta=delta),
                                      delta=delta, target=target))
        learned_best = best_of(rows)
        if learned_best is not None:
            trav = learned_best["traversal"]
            lkw = dict(bkw, traversal=trav, rerank=trav != "f32",
                       mlp=dict(cands)[learned_best["target"]], probe_hops=args.probe_hops,
                       mlp_target=1 if learned_best["target"] == "hops" else 0,
                       mlp_delta=learned_best["delta"])

    # ---- operating point and timed region -----------------------------------------
    if lkw is not None:
        mode, ef, kw, best = "learned_batched", args.ef_max, lkw, learned_best
    elif fixed_best is not None and fixed_best["recall"] >= TARGET_RECALL:
        mode, ef, kw, best = "fixed_batched", fixed_best["ef"], dict(bkw), fixed_best
    else:
        mode, ef, kw, best = "plain_f32", plain_best["ef"], dict(plain_kw), plain_best
    log(f"operating point: {mode} {best}")
    for _ in range(args.warmup):
        ix.search_ex(Q, l, r, k, ef, ids=ids, dists=dists, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ix.search_ex(Q, l, r, k, ef, ids=ids, dists=dists, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1000.0 / args.steps
    qps = nq / (ms_per_step / 1000.0)
    rec_timed = recall(ids, dists)
    # float32 distances returned against float64 ones over the returned points
    samp = np.arange(0, nq, max(1, nq // 500))
    ids_h, d_h = ids[samp].cpu().numpy(), dists[samp].cpu().numpy()
    rel = []
    for i, qi in enumerate(samp):
        ok = ids_h[i] >= 0
        diff = X[ids_h[i][ok]].astype(np.float64) - w["Q"][qi].astype(np.float64)
        d64 = (diff * diff).sum(1)
        rel.append(np.abs(d_h[i][ok].astype(np.float64) - d64) / np.maximum(d64, 1e-30))
    rel = np.concatenate(rel) if rel else np.zeros(1)
    dist_err = {"max_rel": float(rel.max()), "mean_rel": float(rel.mean()),
                "queries": int(len(samp))}

    # ---- roofline of the dominant kernel (graph search over the wide queries) --------
    skw = {kk: v for kk, v in kw.items() if kk not in ("router_threshold", "use_graph")}
    thr = kw.get("router_threshold", 0)
    wide = (width >= thr) if thr else torch.ones_like(width, dtype=torch.bool)
    Qw, lw, rw = Q[wide].contiguous(), l[wide].contiguous(), r[wide].contiguous()
    nw = Qw.shape[0]
    tr = esg.trace_tensor(nw, dev)
    m_part = np.full((nw, 2), ef, np.int64)
    if skw.get("mlp") is not None and skw.get("mlp_target", 0) == 0:
        feat = torch.full((nw, 2, 16), float("nan"), device=dev)
        ix.search_ex(Qw, lw, rw, k, ef, trace=tr, feat_out=feat, **skw)
        fe = feat[:, :, 13].cpu().numpy()
        m_part = np.where(np.isnan(fe), ef, fe).astype(np.int64)
    else:
        ix.search_ex(Qw, lw, rw, k, ef, trace=tr, **skw)
    torch.cuda.synchronize()
    trace = esg.decode_trace(tr)
    elem = {"bf16": 2.0, "fp8": 1.0 + 4.0 / d}.get(skw.get("traversal"), 4.0)
    alg_bytes = algorithmic_bytes(trace, d, info["degree"], k, m_part, elem,
                                  skw.get("rerank", False))
    iw = torch.empty((nw, k), dtype=torch.int64, device=dev)
    dw = torch.empty((nw, k), dtype=torch.float32, device=dev)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for i in range(args.steps):
        starts[i].record()
        ix.search_ex(Qw, lw, rw, k, ef, ids=iw, dists=dw, **skw)
        ends[i].record()
    torch.cuda.synchronize()
    kern_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
    achieved = alg_bytes / (kern_ms / 1000.0) / 1e9
    traffic_key = {kk: kw.get(kk) for kk in ("traversal", "router_threshold", "hash_cap",
                                              "mlp_target", "mlp_delta", "probe_hops")}
    traffic_key.update(ef=ef, workload=args.workload, nq=nw, n=n, learned=kw.get("mlp") is not None)
    traffic = stored_traffic(traffic_key)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oix = oracle.read_index(path)
        done, el, chunk = 0, 0.0, 1000
        while done < nq and el < args.cpu_seconds:
            m = min(chunk, nq - done)
            s0 = time.perf_counter()
            oracle.query_batch(oix, w["Q"][done:done + m], w["l"][done:done + m],
                               w["r"][done:done + m], k, plain_best["ef"])
            el += time.perf_counter() - s0
            done += m
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": round(done / el, 1), "unit": "queries/s", "cores": cores, "kind": "oracle",
               "sample": f"first {done} of the {nq} queries (chunks of {chunk} until "
                         f"{args.cpu_seconds:.0f}s), plain float32 search at the plain point "
                         f"ef={plain_best['ef']}, OpenMP over queries; {el:.1f}s"}
        log(f"cpu oracle {done / el:,.0f} q/s on {cores} cores over {done} queries")

    wl = {2: f"deep-shaped N={n} d={d} unit-norm, {nq} queries, widths log-uniform 10..N, k={k}",
          1: f"sift-shaped N={n} d={d} uint8-valued, {nq} queries, 11 width buckets 2^-b*N, k={k}",
          3: f"embedding-shaped N={n} d={d} unit-norm, {nq} queries, 13 width buckets 2^-b*N, "
             f"k={k}"}[cid]
    out = {
        "metric": "QPS at recall@10>=0.95, learned+batched vs plain search, 1 MI355X; HBM GB/s"
                  if k == 10 else f"QPS at recall@{k}>=0.95, 1 MI355X; HBM GB/s",
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16+f32", "fp8": "fp8+f32"}.get(kw.get("traversal"), "f32"),
        "data": "synthetic",
        "config": {"workload": wl, "variant": mode, f"recall_at_{k}": round(rec_timed, 5),
                   "traversal": kw.get("traversal", "f32"), "distance_error_vs_f64": dist_err,
                   "ef": ef, "delta": best.get("delta"), "target": best.get("target"),
                   "router_threshold": kw.get("router_threshold", 0),
                   "hash_cap": kw.get("hash_cap", 0), "probe_hops": args.probe_hops,
                   "leaf": info["leaf"], "degree": info["degree"], "n_depth": info["n_depth"]},
        "plain_f32": plain_best,
        "fixed_batched": fixed_best,
        "learned_batched": learned_best,
        "speedup_vs_plain": round(qps / plain_best["qps"], 3),
        "learned_gain_vs_fixed": (round(learned_best["qps"] / fixed_best["qps"], 3)
                                  if learned_best and fixed_best else None),
        "training": train_info,
        "sweep": sweep,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "search_kernel", "kernel_ms": round(kern_ms, 4),
                     "queries_per_launch": int(nw), "alg_bytes_per_launch": alg_bytes,
                     "traffic_key": traffic_key},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ix.free()


if __name__ == "__main__":
    main()
