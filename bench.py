#!/usr/bin/env python3
"""Benchmark: QPS at recall@10 >= 0.95 on one MI355X, learned + batched +
bfloat16 search against the plain float32 fixed-ef search.

Default workload (--workload deep): DEEP-shaped batched mixed ranges,
N = 1,000,000 unit-norm vectors in d = 96 (256-centre mixture), attribute =
random permutation, 100,000 queries with range widths log-uniform over
[10, N], k = 10.  The synthetic set stands in for DEEP1M.  --workload sift
runs the SIFT-shaped set (1M x 128 uint8-valued, 10,000 queries in 11
width buckets); --workload embedding the embedding-shaped set at full size
(2M x 768 unit-norm, 20,000 queries in 13 width buckets, k = 100) with
FP8, bfloat16 and float32 traversal (embedding_eval).  The index is built
on the device (the host builder writes the same file).

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
                     of 200,000 separate training queries (GPU kernels);
                     beams chosen before the search are trained for each
                     beam cap in --ef-max (default 24 and 32), the probe
                     forms for the largest.
Every form's setting (its ef, or the network's calibration offset delta)
is chosen on a held-out calibration set: 50,000 queries of the same shape
from their own seed streams (7000+c for vectors, 8000+c for ranges), as the
cheapest setting whose calibration recall reaches 0.95 plus a margin of
three standard errors of that mean (sd of the per-query recall over the
square root of 50,000: about 0.002).  Recall and QPS are
then measured on the evaluation queries.  K steps of the fastest form whose
evaluation recall is >= 0.95 are timed and give `value`; the others are
reported beside it.  One JSON line is printed.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0
TARGET_RECALL = 0.95
CAL_QUERIES = 50_000
CAL_SE = 3.0          # calibration margin in standard errors of the mean recall
# calibration grids: every ef up to 32, then steps of 4 to 64 and of 8 to
# 128 (about 4-12 % of the work per step), and offsets delta in steps of
# 1/16 (2^(1/16): 4.4 % of the beam)
EF_GRID = (list(range(10, 33)) + list(range(36, 65, 4)) + list(range(72, 129, 8)) +
           [160, 192, 224, 256, 320, 384, 512, 768, 1024])
DELTA_GRID = [i / 16.0 for i in range(-16, 9)]
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
                    help="embedding: 2M x 768 unit-norm, k=100, fp8 + f32 rerank evaluation")
    ap.add_argument("--n", type=int, default=None, help="shrink N (default: the full workload)")
    ap.add_argument("--nq", type=int, default=None, help="shrink the query count")
    ap.add_argument("--ntrain", type=int, default=200_000, help="training traces")
    ap.add_argument("--ef-max", type=int, nargs="+", default=[24, 32],
                    help="beam caps of the learned form: beams chosen before the search are "
                         "trained and calibrated for each, the probe forms for the largest")
    ap.add_argument("--probe-hops", type=int, nargs="+", default=[0, 1, 4],
                    help="probe lengths of the learned form (one network each; 0: beams "
                         "chosen before the search from the selection features)")
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
    ap.add_argument("--fanout", type=int, default=2, help="segment-tree fanout of the index")
    ap.add_argument("--host-build", action="store_true",
                    help="build the index with host threads (default: on the device; the "
                         "file is the same)")
    ap.add_argument("--fanout-sweep", action="store_true",
                    help="build the index at fanout 2, 4, 8, 16 and report graph memory, "
                         "build time and plain-search QPS at recall >= 0.95 for the workload's "
                         "range mix and for fixed 2^-5 N ranges; print one JSON line and exit")
    ap.add_argument("--half-bounded", action="store_true",
                    help="half-bounded queries (prefixes and suffixes, widths log-uniform 10..N) "
                         "on the segment-tree index and on the prefix/suffix-chain index (the "
                         "paper's half-bounded index): graph memory and plain-search QPS at "
                         "recall >= 0.95; print one JSON line and exit")
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
    """Hash of the sources the search kernels are compiled from (the
    headers and the per-dimension instantiation unit): a stored traffic
    figure is used only while these are unchanged."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2504_04018_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith(".h") or f == "esg_search_inst.hip":
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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, path, w, k, ef, gt_ids):
    """The oracle as it stands, timed on the host cores: the same float32
    beam search over a bounded sample of the evaluation queries with all
    cores (OpenMP over queries) and with one thread (the paper's
    single-threaded search, Section 5.1), and the float64 brute force of
    Def. 2.2 on a sample.  The brute-force sample also cross-checks the
    GPU's ground truth (the exact scan): tie-aware recall of its top k
    against float64."""
    import ctypes
    import oracle
    oix = oracle.read_index(path)
    gomp = ctypes.CDLL("libgomp.so.1")
    threads = int(gomp.omp_get_max_threads())
    nq = len(w["Q"])
    budget = args.cpu_seconds / 3.0

    def timed(fn, chunk, limit):
        done, el = 0, 0.0
        while done < limit and el < budget:
            m = min(chunk, limit - done)
            s0 = time.perf_counter()
            fn(done, m)
            el += time.perf_counter() - s0
            done += m
        return done, el

    search = lambda s, m: oracle.query_batch(oix, w["Q"][s:s + m], w["l"][s:s + m],
                                             w["r"][s:s + m], k, ef)
    n_mt, t_mt = timed(search, 1000, nq)
    gomp.omp_set_num_threads(1)
    n_st, t_st = timed(search, 100, nq)
    gomp.omp_set_num_threads(threads)
    bf = {}

    def brute(s, m):
        bf[s] = oracle.bruteforce(oix.vec, w["Q"][s:s + m], w["l"][s:s + m], w["r"][s:s + m], k)
    n_bf, t_bf = timed(brute, 200, nq)
    # ground-truth cross-check on the brute-forced sample
    pos_of = np.empty(oix.n, np.int64)
    pos_of[oix.ext_id] = np.arange(oix.n)
    gi = gt_ids[:n_bf]
    found = np.where(gi >= 0, pos_of[np.maximum(gi, 0)], -1)
    gp = np.concatenate([bf[s][0] for s in sorted(bf)])
    gd = np.concatenate([bf[s][1] for s in sorted(bf)])
    rec, strict, _ = oracle.recall(oix.vec, w["Q"][:n_bf], w["l"][:n_bf], w["r"][:n_bf], found,
                                   gp, gd, k)
    log(f"cpu oracle {n_mt / t_mt:,.0f} q/s on {threads} threads, {n_st / t_st:,.0f} q/s on one; "
        f"float64 brute force {n_bf / t_bf:,.1f} q/s; scan ground truth vs float64: {rec}")
    return {"value": round(n_mt / t_mt, 1), "unit": "queries/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"first {n_mt} of the {nq} evaluation queries (chunks of 1000, about "
                      f"{budget:.0f}s), the same float32 beam search at the plain point "
                      f"ef={ef}, OpenMP over queries; {t_mt:.1f}s",
            "single_thread": {"value": round(n_st / t_st, 1), "unit": "queries/s",
                              "sample": f"first {n_st} queries, one thread, {t_st:.1f}s"},
            "bruteforce_f64": {"value": round(n_bf / t_bf, 2), "unit": "queries/s",
                               "cores": threads, "seconds": round(t_bf, 2),
                               "sample": f"first {n_bf} queries, exact float64 filtered k-NN"},
            "gt_check": {"queries": int(n_bf), "recall_of_scan_vs_f64": rec,
                         "strict": strict}}


def load_index(args, cid, w, fanout, layout="tree"):
    import paper_2504_04018_amd as esg
    import synth
    os.makedirs(args.cache_dir, exist_ok=True)
    n = w["n"]
    tag = synth.sha256_of(w["X"][:1000], w["attr"][:1000])[:12]
    path = os.path.join(args.cache_dir,
                        f"{args.workload}_{n}_R{w['degree']}_f{fanout}_{layout}_{tag}.esgi")
    build_s = None
    if not os.path.exists(path):
        t0 = time.time()
        esg.build_index(w["X"], w["attr"].astype(np.float64), path + ".tmp", degree=w["degree"],
                        leaf=w["leaf"], ef_construction=w["ef_construction"], verbose=True,
                        fanout=fanout, layout=layout, device=None if args.host_build else 0)
        os.replace(path + ".tmp", path)
        build_s = time.time() - t0
        log(f"index (fanout {fanout}, {layout}) built on the "
            f"{'host' if args.host_build else 'device'} in {build_s:.1f}s")
    return path, build_s


class Bench:
    """Evaluation and calibration query sets with their exact answers, and
    the measurement of one setting on each."""

    def __init__(self, args, ix, w, wc, dev):
        import torch
        from paper_2504_04018_amd import learned
        self.args, self.ix, self.k = args, ix, w["k"]
        self.dev = dev
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.Q, self.l, self.r = t(w["Q"]), t(w["l"]), t(w["r"])
        self.Qc, self.lc, self.rc = t(wc["Q"]), t(wc["l"]), t(wc["r"])
        self.width, self.widthc = self.r - self.l + 1, self.rc - self.lc + 1
        t0 = time.time()
        self.gt_ids, self.gt_d = learned.exact_answers(ix, self.Q, self.l, self.r, self.k)
        _, self.gt_dc = learned.exact_answers(ix, self.Qc, self.lc, self.rc, self.k)
        torch.cuda.synchronize()
        log(f"exact ground truth (MFMA scan) of {len(self.Q)} + {len(self.Qc)} queries in "
            f"{time.time() - t0:.1f}s")
        self.nq = len(self.Q)
        self.ids = torch.empty((self.nq, self.k), dtype=torch.int64, device=dev)
        self.dists = torch.empty((self.nq, self.k), dtype=torch.float32, device=dev)
        self.sweep = []

    def recall(self, ids, dists, cal=False):
        from paper_2504_04018_amd import learned
        gt, wd = (self.gt_dc, self.widthc) if cal else (self.gt_d, self.width)
        return float(learned.per_query_recall(ids, dists, gt, wd, self.k).mean().item())

    def cal_recall(self, ef, kw, with_se=False):
        from paper_2504_04018_amd import learned
        kw = {kk: v for kk, v in kw.items() if kk != "use_graph"}
        ids, dists = self.ix.search_ex(self.Qc, self.lc, self.rc, self.k, ef, **kw)
        per = learned.per_query_recall(ids, dists, self.gt_dc, self.widthc, self.k)
        mean = float(per.mean().item())
        if with_se:
            return mean, float(per.std().item()) / math.sqrt(per.numel())
        return mean

    def qps(self, ef, kw):
        from paper_2504_04018_amd import autotune
        sec = autotune.time_call(lambda: self.ix.search_ex(self.Q, self.l, self.r, self.k, ef,
                                                           ids=self.ids, dists=self.dists, **kw),
                                 self.args.reps)
        return self.nq / sec

    def evaluate(self, variant, ef, kw, cal_rec, **extra):
        self.ix.search_ex(self.Q, self.l, self.r, self.k, ef, ids=self.ids, dists=self.dists, **kw)
        rec = self.recall(self.ids, self.dists)
        q = self.qps(ef, kw)
        row = dict(variant=variant, ef=ef, traversal=kw.get("traversal", "f32"),
                   cal_recall=round(cal_rec, 5), recall=round(rec, 5), qps=round(q, 1), **extra)
        self.sweep.append(row)
        log(f"{variant} ef={ef} {extra} calibration recall={cal_rec:.4f} "
            f"evaluation recall={rec:.4f} qps={q:,.0f}")
        return row

    def pick(self, candidates):
        """First candidate (cheapest first) whose calibration recall reaches
        the target plus CAL_SE standard errors; each candidate's function
        returns (mean recall, standard error).  Returns (value, recall)."""
        last = None
        for val, fn in candidates:
            rec, se = fn()
            last = (val, rec)
            if rec >= TARGET_RECALL + CAL_SE * se:
                return last
        return last


def embedding_eval(args, dev):
    """Embedding-shaped set at full size (the default N = 2,000,000 unit-norm
    rows in d = 768, 512-centre mixture; 20,000 queries with range widths
    floor(N 2^-b), b = 0..12; k = 100): the index is built on the device,
    traversal in FP8 e4m3 (per-vector scale) with float32 rerank, bfloat16
    with rerank, and float32, each at its cheapest ef whose recall@100 on
    5,000 held-out calibration queries reaches 0.95 plus three standard
    errors.  Reports recall@100 against the exact scan (itself checked
    against float64 brute force on a sample), QPS, the returned distances'
    error against float64, and the search kernel's HBM roofline."""
    import torch
    import paper_2504_04018_amd as esg
    import synth
    t0 = time.time()
    w = synth.make_workload(3, n=args.n, nq=args.nq)
    wc = synth.make_workload(3, n=args.n, nq=5000, query_stream=7000, range_stream=8000)
    del wc["X"]
    n, d, k = w["n"], w["d"], w["k"]
    nq = len(w["Q"])
    log(f"workload {w['name']} n={n} d={d} nq={nq} generated in {time.time() - t0:.1f}s")
    path, build_s = load_index(args, 3, w, 2)
    X = w.pop("X")
    ix = esg.Index(path, 0)
    ix.add_storage("fp8")
    ix.add_storage("bf16")
    ix.reserve(max(nq, 50_000), 4_500_000)
    info = ix.info()
    B = Bench(args, ix, w, wc, dev)
    # the exact scan's answers against float64 brute force on a sample
    pos_ext = np.argsort(w["attr"], kind="stable")         # position -> external id
    samp = np.linspace(0, nq - 1, 24).astype(np.int64)
    gt_ids = B.gt_ids.cpu().numpy()
    hit = tot = 0
    for qi in samp:
        lo, hi = int(w["l"][qi]), int(w["r"][qi])
        q = w["Q"][qi].astype(np.float64)
        dd = np.empty(hi - lo + 1)
        for a in range(lo, hi + 1, 100_000):
            b = min(hi + 1, a + 100_000)
            diff = X[pos_ext[a:b]].astype(np.float64) - q
            dd[a - lo:b - lo] = np.einsum("ij,ij->i", diff, diff)
        kk = min(k, hi - lo + 1)
        kth = np.partition(dd, kk - 1)[kk - 1]
        g = gt_ids[qi][gt_ids[qi] >= 0]
        diff = X[g].astype(np.float64) - q
        hit += min(kk, int((np.einsum("ij,ij->i", diff, diff) <= kth).sum()))
        tot += kk
    gt_check = {"queries": int(len(samp)), "recall_of_scan_vs_f64": hit / tot}
    log(f"scan ground truth vs float64 on {len(samp)} queries: {hit / tot}")

    efs = [100, 112, 128, 160, 192, 256, 320, 384, 512, 640, 768, 1024]
    forms = []
    for trav in ["fp8", "bf16", "f32"]:
        kw = dict(traversal=trav, rerank=trav != "f32")
        ef, cal = B.pick([(e, lambda e=e: B.cal_recall(e, kw, with_se=True)) for e in efs])
        forms.append((B.evaluate(trav, ef, kw, cal), kw))
    train_info = None
    if not args.plain_only:
        # learned beam width chosen before the search, FP8 + rerank, trained
        # on traces of this shape's own training queries: a query's label is
        # the smallest beam of the grid whose top 100 reaches recall 0.97
        from paper_2504_04018_amd import learned
        ntr = min(args.ntrain, 50_000)
        wt = synth.make_workload(3, n=args.n, nq=ntr, query_stream=5000, range_stream=6000)
        del wt["X"]
        tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        Qt, lt, rt = tt(wt["Q"]), tt(wt["l"]), tt(wt["r"])
        _, gt_dt = learned.exact_answers(ix, Qt, lt, rt, k)
        lkw = dict(traversal="fp8", rerank=True)
        nets = []
        train_info = {}
        for cap in (112, 128):     # the beam cap is calibrated like the offset
            t2 = time.time()
            grid = [e for e in (100, 104, 112, 120, 128) if e <= cap]
            F, T = learned.traces(ix, Qt, lt, rt, k, grid, cap, 0, lkw, gt_dt, label_recall=0.97)
            params, hist = learned.train(F, T)
            train_info[f"cap{cap}"] = dict(
                traces=int(F.shape[0]), queries=ntr, first_mse=round(hist[0], 4),
                final_mse=round(hist[-1], 4), seconds=round(time.time() - t2, 1))
            log(f"learned (beams before the search, cap {cap}): {train_info[f'cap{cap}']}")
            nets.append((cap, params))
            del F, T
        del Qt, lt, rt, gt_dt
        for cap, params in nets:
            kw = dict(lkw, mlp=params, probe_hops=0)
            dl, cal = B.pick([(dv, (lambda dv=dv, cap=cap: B.cal_recall(
                cap, dict(kw, mlp_delta=dv), True))) for dv in DELTA_GRID])
            kw["mlp_delta"] = dl
            forms.append((B.evaluate("learned_fp8", cap, kw, cal, delta=dl), kw))
    ok = [f for f in forms if f[0]["recall"] >= TARGET_RECALL]
    best, kw = max(ok or forms, key=lambda f: f[0]["qps"])
    ef = best["ef"]
    Q, l, r = B.Q, B.l, B.r
    ids, dists = B.ids, B.dists
    for _ in range(args.warmup):
        ix.search_ex(Q, l, r, k, ef, ids=ids, dists=dists, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ix.search_ex(Q, l, r, k, ef, ids=ids, dists=dists, **kw)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1000.0 / args.steps
    qps = nq / (ms_per_step / 1000.0)
    rec_timed = B.recall(ids, dists)
    # distances returned against float64 over the returned points
    rows = np.arange(0, nq, max(1, nq // 400))
    ids_h, d_h = ids[rows].cpu().numpy(), dists[rows].cpu().numpy()
    rel = []
    for i, qi in enumerate(rows):
        ok_ = ids_h[i] >= 0
        diff = X[ids_h[i][ok_]].astype(np.float64) - w["Q"][qi].astype(np.float64)
        d64 = (diff * diff).sum(1)
        rel.append(np.abs(d_h[i][ok_].astype(np.float64) - d64) / np.maximum(d64, 1e-30))
    rel = np.concatenate(rel)
    dist_err = {"max_rel": float(rel.max()), "mean_rel": float(rel.mean()), "queries": len(rows)}
    # roofline of the search kernel at the operating point (with a learned
    # form, its beams passed in so that the search kernel is timed alone)
    tr = esg.trace_tensor(nq, dev)
    m_part = np.full((nq, 2), ef, np.int64)
    tkw = kw
    if kw.get("mlp") is not None:
        feat = torch.full((nq, 2, 16), float("nan"), device=dev)
        ix.search_ex(Q, l, r, k, ef, trace=tr, feat_out=feat, **kw)
        fe = feat[:, :, 13].cpu().numpy()
        m_part = np.where(np.isnan(fe), ef, fe).astype(np.int64)
        tkw = {kk: v for kk, v in kw.items() if kk not in ("mlp", "probe_hops", "mlp_delta")}
        tkw["part_ef"] = torch.from_numpy(m_part.astype(np.int32)).to(dev)
    else:
        ix.search_ex(Q, l, r, k, ef, trace=tr, **kw)
    torch.cuda.synchronize()
    trace = esg.decode_trace(tr)
    elem = {"bf16": 2.0, "fp8": 1.0 + 4.0 / d}.get(kw["traversal"], 4.0)
    alg_bytes = algorithmic_bytes(trace, d, info["degree"], k, m_part, elem, kw["rerank"])
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    for s_, e_ in ev:
        s_.record()
        ix.search_ex(Q, l, r, k, ef, ids=ids, dists=dists, **tkw)
        e_.record()
    torch.cuda.synchronize()
    kern_ms = float(np.mean([s_.elapsed_time(e_) for s_, e_ in ev]))
    achieved = alg_bytes / (kern_ms / 1000.0) / 1e9
    tkey = {"traversal": kw["traversal"], "ef": ef, "learned": kw.get("mlp") is not None,
            "mlp_delta": kw.get("mlp_delta"), "workload": "embedding", "nq": nq, "n": n}
    out = {
        "metric": f"QPS at recall@{k}>=0.95, 1 MI355X; HBM GB/s",
        "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16": "bf16+f32", "fp8": "fp8+f32"}.get(kw["traversal"], "f32"),
        "data": "synthetic",
        "config": {"workload": f"embedding-shaped N={n} d={d} unit-norm, {nq} queries, 13 width "
                               f"buckets 2^-b*N, k={k}", "traversal": kw["traversal"], "ef": ef,
                   f"recall_at_{k}": round(rec_timed, 5), "distance_error_vs_f64": dist_err,
                   "fanout": info["fanout"], "leaf": info["leaf"], "degree": info["degree"],
                   "n_depth": info["n_depth"], "device_bytes": info["device_bytes"],
                   "index_build_s_device": None if build_s is None else round(build_s, 1),
                   "gt_check": gt_check, "delta": best.get("delta"), "training": train_info},
        "forms": [f[0] for f in forms],
        "sweep": B.sweep,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": stored_traffic(tkey), "kernel": "search_kernel",
                     "kernel_ms": round(kern_ms, 4), "queries_per_launch": nq,
                     "alg_bytes_per_launch": alg_bytes, "traffic_key": tkey},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    ix.free()


def fanout_sweep(args, cid, dev):
    """Graph memory, build time and plain float32 QPS at recall >= 0.95 per
    fanout (Section 4.2, Extensions; the paper's Exp-6)."""
    import torch
    import paper_2504_04018_amd as esg
    from paper_2504_04018_amd import learned
    import synth
    w = synth.make_workload(cid, n=args.n, nq=args.nq)
    wc = synth.make_workload(cid, n=args.n, nq=CAL_QUERIES, query_stream=7000, range_stream=8000)
    del wc["X"]
    n, k = w["n"], w["k"]
    lf, rf = synth.fixed_width_ranges(n, len(w["Q"]), 2.0 ** -5, 9000 + cid)
    lfc, rfc = synth.fixed_width_ranges(n, CAL_QUERIES, 2.0 ** -5, 9500 + cid)
    rows = []
    for f in (2, 4, 8, 16):
        path, build_s = load_index(args, cid, w, f)
        ix = esg.Index(path, 0)
        ix.add_storage("bf16")
        ix.reserve(max(len(w["Q"]), CAL_QUERIES), 4_500_000)
        info = ix.info()
        row = {"fanout": f, "n_depth": info["n_depth"],
               "graph_bytes": int(info["n_depth"] * n * info["degree"] * 4),
               "build_s": None if build_s is None else round(build_s, 1)}
        for name, (l, r, lc, rc) in {"mix": (w["l"], w["r"], wc["l"], wc["r"]),
                                     "fixed_2^-5N": (lf, rf, lfc, rfc)}.items():
            wv = dict(w, l=l, r=r)
            wcv = dict(wc, l=lc, r=rc)
            b = Bench(args, ix, wv, wcv, dev)
            ef, cr = b.pick([(ef, (lambda e=ef: b.cal_recall(e, {}, True)))
                             for ef in EF_GRID if ef >= k])
            ev = b.evaluate(f"plain_f32_f{f}_{name}", ef, {}, cr)
            row[name] = {"ef": ef, "cal_recall": ev["cal_recall"], "recall": ev["recall"],
                         "qps": ev["qps"]}
            del b
            torch.cuda.empty_cache()
        rows.append(row)
        ix.free()
        log(f"fanout {f}: {row}")
    print(json.dumps({"fanout_sweep": rows, "workload": w["name"], "n": n, "k": k,
                      "queries": len(w["Q"]), "calibration_queries": CAL_QUERIES}), flush=True)


def half_bounded(args, cid, dev):
    """Half-bounded queries on the two index layouts (Section 4.1 against
    Section 4.2): graph memory, build time, plain float32 QPS at recall >=
    0.95 (ef calibrated on held-out half-bounded queries)."""
    import torch
    import paper_2504_04018_amd as esg
    import synth
    w = synth.make_workload(cid, n=args.n, nq=args.nq)
    wc = synth.make_workload(cid, n=args.n, nq=CAL_QUERIES, query_stream=7000, range_stream=8000)
    del wc["X"]
    n, k = w["n"], w["k"]
    w["l"], w["r"] = synth.half_bounded_ranges(n, len(w["Q"]), 10, 9100 + cid)
    wc["l"], wc["r"] = synth.half_bounded_ranges(n, CAL_QUERIES, 10, 9600 + cid)
    rows = []
    for layout in ("tree", "chain"):
        path, build_s = load_index(args, cid, w, 2, layout)
        ix = esg.Index(path, 0)
        ix.add_storage("bf16")
        ix.reserve(max(len(w["Q"]), CAL_QUERIES), 4_500_000)
        info = ix.info()
        rows_per = (info["n_depth"] * n if layout == "tree"
                    else 2 * sum(_chain_sizes(n, info["leaf"], 2)))
        b = Bench(args, ix, w, wc, dev)
        ef, cr = b.pick([(e, (lambda e=e: b.cal_recall(e, {}, True))) for e in EF_GRID if e >= k])
        ev = b.evaluate(f"plain_f32_{layout}", ef, {}, cr)
        rows.append({"layout": layout, "n_depth": info["n_depth"],
                     "graph_bytes": int(rows_per * info["degree"] * 4),
                     "build_s": None if build_s is None else round(build_s, 1),
                     "ef": ef, "cal_recall": ev["cal_recall"], "recall": ev["recall"],
                     "qps": ev["qps"]})
        log(f"half-bounded {layout}: {rows[-1]}")
        del b
        ix.free()
        torch.cuda.empty_cache()
    print(json.dumps({"half_bounded": rows, "workload": w["name"], "n": n, "k": k,
                      "queries": len(w["Q"]), "calibration_queries": CAL_QUERIES}), flush=True)


def _chain_sizes(n, leaf, base):
    out, s = [], n
    while s - 1 >= leaf:
        out.append(s)
        if s == 1:
            break
        s = -(-s // base)
    return out


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
    if cid == 3 and not (args.fanout_sweep or args.half_bounded or args.scan_only):
        embedding_eval(args, dev)
        return
    if args.fanout_sweep:
        fanout_sweep(args, cid, dev)
        return
    if args.half_bounded:
        half_bounded(args, cid, dev)
        return
    t0 = time.time()
    w = synth.make_workload(cid, n=args.n, nq=args.nq)
    wc = synth.make_workload(cid, n=args.n, nq=CAL_QUERIES, query_stream=7000, range_stream=8000)
    del wc["X"]
    n, d, k = w["n"], w["d"], w["k"]
    nq = len(w["Q"])
    log(f"workload {w['name']} n={n} d={d} nq={nq} (+{CAL_QUERIES} calibration) generated in "
        f"{time.time() - t0:.1f}s")
    path, _ = load_index(args, cid, w, args.fanout)
    X = w.pop("X")                        # kept for the float64 distance check
    ix = esg.Index(path, 0)
    ix.add_storage("bf16")
    if cid == 3:
        ix.add_storage("fp8")
    ix.reserve(max(nq, args.ntrain, CAL_QUERIES), 4_500_000)
    info = ix.info()
    B = Bench(args, ix, w, wc, dev)
    Q, l, r, width = B.Q, B.l, B.r, B.width

    if args.scan_only:
        # exact scan: algorithmic flops 2*w*d per query (in-range points only)
        wsum = float((width).sum().item())
        alg_flops = 2.0 * wsum * d
        cap = 64 if k <= 32 else (128 if k <= 64 else 256)
        mr, scan_table = autotune.tune_scan(ix, Q, l, r, k,
                                            sorted({k, 2 * k, 4 * k, cap // 2, cap - 1}),
                                            log=log)
        t_ms, nfb = [], 0
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, nfb = ix.scan(Q, l, r, k, rerank_count=mr)
            torch.cuda.synchronize()
            if i >= args.warmup:
                t_ms.append((time.perf_counter() - t0) * 1000.0)
        ms = float(np.median(t_ms))
        tf = alg_flops / (ms / 1000.0) / 1e12
        print(json.dumps({"scan_only": True, "workload": args.workload, "n": n, "d": d, "nq": nq,
                          "k": k, "ms_per_batch": round(ms, 3), "queries_per_s": round(nq / ms * 1e3),
                          "alg_tflop_per_batch": round(alg_flops / 1e12, 3),
                          "alg_tflops": round(tf, 1), "bf16_peak_tflops": MFMA_BF16_PEAK_TFLOPS,
                          "frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 4), "n_fallback": int(nfb),
                          "rerank_count": mr, "tune": scan_table}))
        return

    def ef_candidates(kw):
        grid = [args.fixed_ef] if args.fixed_ef else [e for e in EF_GRID if e >= k]
        return [(e, (lambda e=e: B.cal_recall(e, kw, True))) for e in grid]

    # ---- plain: float32 traversal, fixed ef -------------------------------------
    plain_kw = dict(traversal="f32")
    ef_p, cr = B.pick(ef_candidates(plain_kw))
    plain_best = B.evaluate("plain_f32", ef_p, plain_kw, cr)

    # ---- batched, fixed ef, autotuned launch settings --------------------------------
    fixed_best = learned_best = train_info = None
    learned_rows = []
    bkw = None
    if not args.plain_only:
        base = dict(use_graph=True)
        grid = {"traversal": [args.traversal] if args.traversal else
                (["fp8", "bf16", "f32"] if cid == 3 else ["bf16", "f32"]),
                "router_threshold": [args.router] if args.router is not None else [0, 512, 2048],
                "hash_cap": [args.hash_cap] if args.hash_cap else [4096, 8192]}

        def measure(kw):
            kw = dict(kw, rerank=kw["traversal"] != "f32")
            return B.cal_recall(ef_p, kw), B.qps(ef_p, kw)
        # knobs that keep the recall of the plain point (within 0.002) may be
        # traded for speed; the beam itself is calibrated afterwards
        tuned, _ = autotune.tune_settings(base, grid, measure, cr - 0.002, log=log)
        tuned["rerank"] = tuned["traversal"] != "f32"
        bkw = {kk: tuned[kk] for kk in ("traversal", "rerank", "use_graph", "router_threshold",
                                         "hash_cap")}
        ef_f, cr = B.pick(ef_candidates(bkw))
        fixed_best = B.evaluate("fixed_batched", ef_f, bkw, cr)

    caps = sorted(c for c in args.ef_max if c >= k)
    if not args.plain_only and not caps:
        log(f"learned form skipped: --ef-max {args.ef_max} < k = {k}")
    elif not args.plain_only:
        # ---- learned: traces of separate training queries, GPU training ------------------
        wt = synth.make_workload(cid, n=n, nq=args.ntrain, query_stream=5000, range_stream=6000)
        del wt["X"]
        tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        Qt, lt, rt = tt(wt["Q"]), tt(wt["l"]), tt(wt["r"])
        _, gt_dt = learned.exact_answers(ix, Qt, lt, rt, k)
        tkw = {kk: v for kk, v in bkw.items() if kk != "use_graph"}
        train_info = {}
        nets = []
        for probe in args.probe_hops:
            for target, grid in (("ef", LABEL_EF_GRID), ("hops", LABEL_HOP_GRID)):
                if (args.target and target != args.target) or (probe == 0 and target == "hops"):
                    continue                 # a stopping step needs a probe
                for cap in (caps if probe == 0 else caps[-1:]):
                    t1 = time.time()
                    g = [v for v in grid if target == "hops" or v <= cap]
                    F, T = learned.traces(ix, Qt, lt, rt, k, g, cap, probe, tkw, gt_dt,
                                          target=target)
                    params, hist = learned.train(F, T)
                    name = f"{target}_probe{probe}" + (f"_cap{cap}" if probe == 0 else "")
                    train_info[name] = dict(
                        traces=int(F.shape[0]), queries=args.ntrain, first_mse=round(hist[0], 4),
                        final_mse=round(hist[-1], 4), seconds=round(time.time() - t1, 2))
                    log(f"learned target={target} probe={probe} cap={cap}: {F.shape[0]} part "
                        f"traces, mse {hist[0]:.3f} -> {hist[-1]:.3f} in {time.time() - t1:.1f}s")
                    nets.append((target, probe, cap, params))
                    del F, T
        del Qt, lt, rt, gt_dt
        travs = [bkw["traversal"]] + ([] if args.traversal else
                                      [t for t in ("bf16", "f32") if t != bkw["traversal"]])
        for target, probe, cap, params in nets:
            for trav in travs:
                kw = dict(bkw, traversal=trav, rerank=trav != "f32", mlp=params,
                          probe_hops=probe, mlp_target=1 if target == "hops" else 0)
                deltas = [args.delta] if args.delta is not None else DELTA_GRID
                dl, cr = B.pick([(dv, (lambda dv=dv, cap=cap: B.cal_recall(
                    cap, dict(kw, mlp_delta=dv), True))) for dv in deltas])
                kw["mlp_delta"] = dl
                row = B.evaluate("learned_batched", cap, kw, cr, delta=dl, target=target,
                                 probe_hops=probe)
                learned_rows.append((row, kw))
        ok = [(rw, kw) for rw, kw in learned_rows if rw["recall"] >= TARGET_RECALL]
        if ok:
            learned_best, lkw = max(ok, key=lambda t: t[0]["qps"])

    # ---- operating point and timed region -----------------------------------------
    forms = [("plain_f32", plain_best["ef"], dict(plain_kw), plain_best)]
    if fixed_best is not None:
        forms.append(("fixed_batched", fixed_best["ef"], dict(bkw), fixed_best))
    if learned_best is not None:
        forms.append(("learned_batched", learned_best["ef"], lkw, learned_best))
    # the learned + batched form is the one the metric names; without it, the
    # fastest form whose evaluation recall reaches the target
    ok = [f for f in forms if f[3]["recall"] >= TARGET_RECALL]
    if learned_best is not None:
        mode, ef, kw, best = forms[-1]
    else:
        mode, ef, kw, best = max(ok or forms[:1], key=lambda f: f[3]["qps"])
    log(f"operating point: {mode} {best}")
    ids, dists = B.ids, B.dists
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
    rec_timed = B.recall(ids, dists)
    # float32 distances returned against float64 ones over the returned points
    samp = np.arange(0, nq, max(1, nq // 500))
    ids_h, d_h = ids[samp].cpu().numpy(), dists[samp].cpu().numpy()
    rel = []
    for i, qi in enumerate(samp):
        ok_ = ids_h[i] >= 0
        diff = X[ids_h[i][ok_]].astype(np.float64) - w["Q"][qi].astype(np.float64)
        d64 = (diff * diff).sum(1)
        rel.append(np.abs(d_h[i][ok_].astype(np.float64) - d64) / np.maximum(d64, 1e-30))
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
    tkw = skw
    if skw.get("mlp") is not None and skw.get("probe_hops", 1) == 0:
        # beams chosen before the search: time the search kernel alone, with
        # the beams the predictor chose passed in (the predictor kernel is
        # timed inside the step above, not here)
        tkw = {kk: v for kk, v in skw.items() if kk not in ("mlp", "probe_hops", "mlp_delta",
                                                             "mlp_target")}
        tkw["part_ef"] = torch.from_numpy(m_part.astype(np.int32)).to(dev)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for i in range(args.steps):
        starts[i].record()
        ix.search_ex(Qw, lw, rw, k, ef, ids=iw, dists=dw, **tkw)
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
        cpu = cpu_baseline(args, path, w, k, plain_best["ef"], B.gt_ids.cpu().numpy())

    wl = {2: f"deep-shaped N={n} d={d} unit-norm, {nq} queries, widths log-uniform 10..N, k={k}",
          1: f"sift-shaped N={n} d={d} uint8-valued, {nq} queries, 11 width buckets 2^-b*N, k={k}",
          3: f"embedding-shaped N={n} d={d} unit-norm, {nq} queries, 13 width buckets 2^-b*N, "
             f"k={k}"}[cid]
    lb16 = [rw_ for rw_, _ in learned_rows if rw_["traversal"] == "bf16"
            and rw_["recall"] >= TARGET_RECALL]
    best16 = max(lb16, key=lambda t: t["qps"]) if lb16 else None
    target = {
        "statement": "learned + batched + bfloat16 beats plain float32 fixed-ef (and fixed-ef "
                     "bfloat16 batched) at recall@10 >= 0.95",
        "learned_bf16_qps": best16["qps"] if best16 else None,
        "learned_bf16_recall": best16["recall"] if best16 else None,
        "beats_plain_f32": bool(best16 and best16["qps"] > plain_best["qps"]),
        "beats_fixed_batched": bool(best16 and fixed_best and best16["qps"] > fixed_best["qps"]),
    }
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
                   "probe_hops": best.get("probe_hops"),
                   "router_threshold": kw.get("router_threshold", 0),
                   "hash_cap": kw.get("hash_cap", 0), "fanout": info["fanout"],
                   "leaf": info["leaf"], "degree": info["degree"], "n_depth": info["n_depth"],
                   "calibration": {"queries": CAL_QUERIES, "query_seed": 7000 + cid,
                                   "range_seed": 8000 + cid, "margin_se": CAL_SE}},
        "plain_f32": plain_best,
        "fixed_batched": fixed_best,
        "learned_batched": learned_best,
        "target": target,
        "speedup_vs_plain": round(qps / plain_best["qps"], 3),
        "learned_gain_vs_fixed": (round(learned_best["qps"] / fixed_best["qps"], 3)
                                  if learned_best and fixed_best else None),
        "training": train_info,
        "sweep": B.sweep,
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
