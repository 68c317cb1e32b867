#!/usr/bin/env python3
"""Benchmark of threshold / symmetric queries over bitmaps on one MI355X.

Default workload ("large"): N = 256 uncompressed bitmaps of r = 2^26 bits
(2 GiB), per-bitmap density log-uniform in [1e-4, 0.5].  One step runs the
workload's query set once: thresholds 2, 16, 128, 255, the interval query
2 <= count <= 10 and parity, each reading all 2 GiB.  Inputs are generated on
the GPU before timing and stay resident in HBM.

Prints one JSON line: logical input GB/s over the timed steps, the roofline of
the dense counter kernel (algorithmic bytes per launch over its mean launch
time, taken with HIP events on the library's stream), and the CPU oracle timed
on a bounded sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=["large", "small", "rle", "serving", "selector"])
    ap.add_argument("--selector-queries", type=int, default=2500)
    ap.add_argument("--selector-train", type=int, default=2000)
    ap.add_argument("--selector-out", default=None,
                    help="directory for the selector's timing dataset and trained weights (not written if unset)")
    ap.add_argument("--serving-queries", type=int, default=20000)
    ap.add_argument("--serving-inflight", type=int, default=4,
                    help="batches in flight at once in the serving client (1..4)")
    ap.add_argument("--serving-shared-stream", action="store_true",
                    help="submit every batch on one stream instead of one stream per slot")
    ap.add_argument("--serving-selector", default="batch", choices=["batch", "train", "single"],
                    help="weights of the serving selector: batch = shipped weights trained on batch-path costs "
                         "(trained here if none are shipped), train = train them here, single = the "
                         "single-query weights")
    ap.add_argument("--serving-train-queries", type=int, default=600)
    ap.add_argument("--serving-eval-queries", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-consumers", action="store_true",
                    help="skip the fused-consumer and weighted timings (profiling runs of the roofline kernel)")
    ap.add_argument("--prune", type=int, default=1,
                    help="threshold pruning in the timed pass (the roofline pass never prunes)")
    ap.add_argument("--no-summaries", action="store_true",
                    help="default workload only: skip the compact RLE, serving and selector summaries")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--record-traffic", metavar="PMC_DIR",
                    help="write profiles/traffic.json from rocprofv3 counter runs under PMC_DIR (no GPU "
                         "work): fetch/, write/, raw/ of the default step, cfetch/, cwrite/, craw/ of "
                         "--copy-calibration, rle_fetch/, rle_write/ of --workload rle")
    return ap.parse_args()


# ------------------------------------------------------------ traffic records
# Sources each record is keyed on: a record counts only while every one of
# them is unchanged (load_traffic compares their hash).
DENSE_SOURCES = ["paper_1402_4073_amd/csrc/tq_dense.hip", "paper_1402_4073_amd/csrc/tq_csa.hpp",
                 "paper_1402_4073_amd/csrc/tq_internal.h", "include/tq.h"]
STEP_SOURCES = DENSE_SOURCES + ["paper_1402_4073_amd/csrc/tq_looped.hip", "paper_1402_4073_amd/csrc/tq_variants.hpp",
                                "paper_1402_4073_amd/csrc/tq_host.hip", "paper_1402_4073_amd/csrc/tq_select.hip",
                                "tqgen/__init__.py", "tqgen/gen.hip"]
RLE_SOURCES = ["paper_1402_4073_amd/csrc/tq_rle.hip", "paper_1402_4073_amd/csrc/tq_csa.hpp",
               "paper_1402_4073_amd/csrc/tq_internal.h", "include/tq.h"]
STEP_QUERIES = ["theta 2", "theta 16", "theta 128", "theta 255", "2 <= count <= 10", "parity"]


def source_sha(sources):
    import hashlib
    return hashlib.sha256(b"".join(open(os.path.join(ROOT, s), "rb").read() for s in sources)).hexdigest()[:16]


def pmc_dispatches(d):
    """(dispatch id, kernel name, {counter: value summed over the device})
    from the counter_collection csv files of one rocprofv3 run."""
    import csv
    import glob
    by = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                k = int(r.get("Dispatch_Id") or r.get("Dispatch_ID"))
                e = by.setdefault(k, {"kernel": r.get("Kernel_Name"), "c": {}})
                e["c"][r["Counter_Name"]] = e["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [(k, by[k]["kernel"], by[k]["c"]) for k in sorted(by)]


def record_traffic(pmc_dir):
    """HBM bytes per launch from FETCH_SIZE / WRITE_SIZE, each scaled by what
    the same counter reads for a plain 1 GiB copy."""
    def mean(v):
        return sum(v) / len(v)
    def copies(sub, ctr):
        return [c[ctr] for _, n, c in pmc_dispatches(os.path.join(pmc_dir, sub)) if "copyBuffer" in n]
    fscale = 1048576.0 / mean(copies("cfetch", "FETCH_SIZE"))
    wscale = 1048576.0 / mean(copies("cwrite", "WRITE_SIZE"))
    raw_copy = mean(copies("craw", "TCC_EA0_RDREQ_sum"))

    def step(sub, ctr):
        return [(n, c[ctr]) for _, n, c in pmc_dispatches(os.path.join(pmc_dir, sub))
                if "looped_kernel" in n or "dense_kernel" in n]
    F, W, R = step("fetch", "FETCH_SIZE"), step("write", "WRITE_SIZE"), step("raw", "TCC_EA0_RDREQ_sum")
    # bench.py --steps 1 --warmup 1 --no-consumers --no-summaries: the pruned step twice (warm-up and
    # timed, six queries each), then the unpruned roofline pass twice
    if not (len(F) == len(W) == len(R) == 24):
        raise SystemExit("expected 24 dense/looped dispatches per run, got %d/%d/%d" % (len(F), len(W), len(R)))
    queries = []
    for i, name in enumerate(STEP_QUERIES):
        fk = mean([F[s * 6 + i][1] for s in (0, 1)])
        wk = mean([W[s * 6 + i][1] for s in (0, 1)])
        rq = mean([R[s * 6 + i][1] for s in (0, 1)])
        kern = F[6 + i][0].replace("void tq::(anonymous namespace)::", "").split("(")[0]
        queries.append({"query": name, "kernel": kern, "fetch_kib": fk, "write_kib": wk, "rdreq": rq,
                        "bytes": int(round(fk * 1024 * fscale + wk * 1024 * wscale))})
    uf = mean([f for _, f in F[12:]])
    uw = mean([w for _, w in W[12:]])
    rec = {}
    rec["dense_kernel<K=9>/large"] = {
        "source_sha": source_sha(DENSE_SOURCES),
        "bytes_per_launch": int(round(uf * 1024 * fscale + uw * 1024 * wscale)),
        "fetch_kib_per_dispatch": round(uf, 2), "write_kib_per_dispatch": round(uw, 2),
        "fetch_scale": fscale, "write_scale": wscale,
        "note": "launches with pruning off (12 dispatches); FETCH_SIZE/WRITE_SIZE (KiB per dispatch) scaled by "
                "what they read for a plain 1 GiB copy; see hbm_counter_calibration.md",
        "sources": DENSE_SOURCES}
    rec["dense_step/large-pruned"] = {
        "source_sha": source_sha(STEP_SOURCES), "bytes_per_query": [q["bytes"] for q in queries],
        "queries": queries, "fetch_scale": fscale, "write_scale": wscale,
        "note": "default step (pruning and Looped on, registered inputs read by cardinality): HBM bytes per "
                "query from FETCH_SIZE and WRITE_SIZE per dispatch, mean of the two steps of the run, scaled "
                "as the dense kernel's",
        "sources": STEP_SOURCES}
    # threshold launches of the tile kernel: compressed inputs only, no consumers, bit planes
    rf = [(n, c["FETCH_SIZE"]) for _, n, c in pmc_dispatches(os.path.join(pmc_dir, "rle_fetch"))
          if "rle_tile_kernel" in n and ", false, false, 1, false, false>" in n]
    rw = [(n, c["WRITE_SIZE"]) for _, n, c in pmc_dispatches(os.path.join(pmc_dir, "rle_write"))
          if "rle_tile_kernel" in n and ", false, false, 1, false, false>" in n]
    if not rf or len(rf) != len(rw):
        raise SystemExit("RLE threshold dispatches: %d fetch, %d write" % (len(rf), len(rw)))
    f, w = mean([v for _, v in rf]), mean([v for _, v in rw])
    rec["rle_tile_kernel/rle-thresholds"] = {
        "source_sha": source_sha(RLE_SOURCES),
        "bytes_per_launch": int(round(f * 1024 * fscale + w * 1024 * wscale)),
        "fetch_kib_per_dispatch": round(f, 1), "write_kib_per_dispatch": round(w, 1),
        "fetch_scale": fscale, "write_scale": wscale,
        "note": "threshold launches (thetas 2, 64, 256 with RLE and dense output, %d dispatches averaged); same "
                "scaling as the dense kernel" % len(rf),
        "sources": RLE_SOURCES}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({"copy_fetch_scale": fscale, "copy_write_scale": wscale, "copy_rdreq": raw_copy,
                      "dense_bytes_per_launch": rec["dense_kernel<K=9>/large"]["bytes_per_launch"],
                      "step_bytes": sum(q["bytes"] for q in queries),
                      "rle_bytes_per_launch": rec["rle_tile_kernel/rle-thresholds"]["bytes_per_launch"]}))


def copy_calibration():
    """A plain copy of known size: 1 GiB read + 1 GiB written per launch."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.int64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_launch": 1 << 30,
                                           "bytes_written_per_launch": 1 << 30, "launches": 3}}))


def load_traffic(kernel_key: str, field: str = "bytes_per_launch"):
    """HBM bytes measured by rocprofv3 counters (profiles/traffic.json): the
    record's `field`, or None if not measured for the current sources of
    that kernel."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not rec or "sources" not in rec:
        return None
    # every source the kernel is compiled from, in the listed order
    try:
        blob = b"".join(open(os.path.join(ROOT, s), "rb").read() for s in rec["sources"])
    except OSError:
        return None
    h = hashlib.sha256(blob).hexdigest()[:16]
    if rec.get("source_sha") != h:
        return None
    return rec.get(field)


def cpu_baseline(pool_rows, n, nwords, r_bits, queries, target_s, threads=None):
    """The oracle as it stands, on a contiguous column sample of every bitmap
    (all of the host's OpenMP threads, or `threads`)."""
    import numpy as np
    import oracle
    if threads:
        oracle.set_threads(threads)
    threads = oracle.max_threads()
    m = 2048
    sample_host = None
    while True:
        cols = np.arange(m, dtype=np.uint64)
        words = np.stack([r[:m].cpu().numpy().view(np.uint64) for r in pool_rows])
        t0 = time.perf_counter()
        for kind, arg in queries:
            if kind == "threshold":
                oracle.threshold_cols(words, cols, r_bits, arg)
            else:
                oracle.symmetric_cols(words, cols, r_bits, arg)
        dt = time.perf_counter() - t0
        sample_host = (m, dt)
        if dt >= target_s or m >= nwords:
            break
        m = int(min(nwords, max(2 * m, m * target_s / max(dt, 1e-3) * 1.1)))
    m, dt = sample_host
    reps = 1
    if dt < target_s:
        # the whole workload took less than the target: repeat it (adaptive
        # repetition, as the paper times its runs)
        reps = max(1, int(target_s / max(dt, 1e-3)))
        t0 = time.perf_counter()
        for _ in range(reps):
            for kind, arg in queries:
                if kind == "threshold":
                    oracle.threshold_cols(words, cols, r_bits, arg)
                else:
                    oracle.symmetric_cols(words, cols, r_bits, arg)
        dt = time.perf_counter() - t0
    in_bytes = reps * len(queries) * n * m * 8
    return {"value": round(in_bytes / dt / 1e9, 4), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d of %d word columns of all %d bitmaps, %d queries x %d passes, %.1f s"
                      % (m, nwords, n, len(queries), reps, dt)}


def bench_rle(args):
    """RLE workload: N=512 Markov bitmaps of r=2^28 bits (ones-runs mean 64,
    zeros-runs mean 4096), canonical streams with checkpoint indexes built by
    the library's encoder before timing; thresholds 2, 64, 256 with canonical
    RLE output."""
    import numpy as np
    import torch
    import tqgen
    from paper_1402_4073_amd import binding as tq

    ms = tqgen.rle_set(3)
    n, nw, r = ms.n, ms.nwords, ms.r_bits
    thetas = tqgen.RLE["thetas"]
    ctx = tq.tq_create(0)
    dense = torch.empty((n, nw), dtype=torch.int64, device="cuda:0")
    for j0 in range(0, n, 64):
        tqgen.fill_gpu(ms, dense[j0:j0 + 64].reshape(-1), first=j0, count=min(64, n - j0))
    rows = [dense[j] for j in range(n)]
    pool, offs, lens, index_pool = tq.encode_pool(ctx, rows, r)
    sample_cols = 1 << 12
    host_sample = np.stack([rw[:sample_cols].cpu().numpy().view(np.uint64) for rw in rows])
    del rows
    del dense
    torch.cuda.empty_cache()
    inputs = [(pool[offs[j]:], lens[j], index_pool[j]) for j in range(n)]
    comp_bytes = sum(lens) * 8
    ntiles = (nw + tq.TQ_RLE_INDEX_STRIDE - 1) // tq.TQ_RLE_INDEX_STRIDE
    index_bytes_read = n * ntiles * 16
    cap = tq.tq_rle_max_words(r)
    out = torch.empty(cap, dtype=torch.int64, device="cuda:0")
    dout = torch.empty(nw, dtype=torch.int64, device="cuda:0")
    ln = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    stream = torch.cuda.Stream(device="cuda:0")
    ev_full, ev_tile = [], []
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            for t in thetas:
                tq.tq_threshold_rle(ctx, inputs, r, t, out, cap, ln, stream)
                tq.tq_threshold_rle_dense(ctx, inputs, r, t, dout, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for t in thetas:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                tq.tq_threshold_rle(ctx, inputs, r, t, out, cap, ln, stream)
                b.record(stream)
                ev_full.append((a, b))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # r0 / r1 bracket the tile launches of steps 2..K (back to back on the stream)
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for s in range(args.steps):
            if s == 1:
                r0.record(stream)
            for t in thetas:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                tq.tq_threshold_rle_dense(ctx, inputs, r, t, dout, stream)
                b.record(stream)
                ev_tile.append((a, b))
        r1.record(stream)
        torch.cuda.synchronize()
    # symmetric functions over the same compressed inputs (canonical RLE output)
    sym = {"parity": tq.truth_parity(n), "2<=count<=10": tq.truth_interval(n, 2, 10)}
    sym_ms = {}
    with torch.cuda.stream(stream):
        for name, t in sym.items():
            tq.tq_symmetric_rle(ctx, inputs, r, t, out, cap, ln, stream)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(args.steps):
                tq.tq_symmetric_rle(ctx, inputs, r, t, out, cap, ln, stream)
            b.record(stream)
            torch.cuda.synchronize()
            sym_ms[name] = round(a.elapsed_time(b) / args.steps, 4)
    # the same queries with no checkpoint index supplied: the library builds
    # the missing indexes (one launch, one wave per stream) into its
    # workspace before the tile kernel
    noidx = [(pool[offs[j]:], lens[j], None) for j in range(n)]
    noidx_ms = {}
    with torch.cuda.stream(stream):
        for t in thetas:
            tq.tq_threshold_rle_dense(ctx, noidx, r, t, dout, stream)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(args.steps):
                tq.tq_threshold_rle_dense(ctx, noidx, r, t, dout, stream)
            b.record(stream)
            torch.cuda.synchronize()
            noidx_ms[str(t)] = round(a.elapsed_time(b) / args.steps, 4)
    # fused consumer: the count of each threshold result, nothing stored
    count_ms = {}
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    with torch.cuda.stream(stream):
        for t in thetas:
            tq.tq_threshold_rle_fused(ctx, inputs, r, t, None, None, cnt, stream)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(args.steps):
                tq.tq_threshold_rle_fused(ctx, inputs, r, t, None, None, cnt, stream)
            b.record(stream)
            torch.cuda.synchronize()
            count_ms[str(t)] = round(a.elapsed_time(b) / args.steps, 4)
    st = tq.tq_ctx_check(ctx, stream)
    if st != 0:
        raise RuntimeError("device error: %s" % tq.status_string(st))
    elapsed = t1 - t0
    q = len(thetas)
    full_ms = [a.elapsed_time(b) for a, b in ev_full]
    tile_ms = [a.elapsed_time(b) for a, b in ev_tile]
    uncompressed = n * nw * 8
    alg = comp_bytes + index_bytes_read + nw * 8
    # mean launch, bounded from above by an event pair around every launch and
    # by the span of steps 2..K over their launches; the smaller bound is used
    tile_pair_s = sum(tile_ms) / len(tile_ms) / 1e3
    tile_span_s = r0.elapsed_time(r1) / ((args.steps - 1) * len(thetas)) / 1e3 if args.steps > 1 else tile_pair_s
    tile_s = min(tile_pair_s, tile_span_s)
    rec = {
        "metric": "uncompressed-equivalent input GB/s per RLE threshold query (RLE in, canonical RLE out)",
        "value": round(q * uncompressed * args.steps / elapsed / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64 bitwise", "data": "synthetic (seeded two-state Markov chain, encoded on the GPU)",
        "config": {"workload": "RLE: N=512 bitmaps, r=2^28 bits, Markov runs mean 64 (ones) / 4096 (zeros); "
                               "thresholds 2, 64, 256; canonical RLE output",
                   "compressed_bytes": comp_bytes, "uncompressed_bytes_per_query": uncompressed},
        "compressed_input_GBps": round(q * comp_bytes * args.steps / elapsed / 1e9, 2),
        "per_query_ms": [round(sum(full_ms[i::q]) / args.steps, 4) for i in range(q)],
        "tile_kernel_ms": [round(sum(tile_ms[i::q]) / args.steps, 4) for i in range(q)],
        "symmetric_query_ms": sym_ms,
        "count_only_query_ms": count_ms,
        "no_index_dense_query_ms": noidx_ms,
        "roofline": {"bound": "hbm", "achieved": round(alg / tile_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(alg / tile_s / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic("rle_tile_kernel/rle-thresholds"),
                     "kernel": "rle_tile_kernel (bit_length(theta - 1) exact planes and a sticky one: theta 2: 2 planes; 64: 7; 256: 9)",
                     "mean_launch_us": round(tile_s * 1e6, 2),
                     "mean_launch_us_event_pair_each": round(tile_pair_s * 1e6, 2),
                     "mean_launch_us_span": round(tile_span_s * 1e6, 2),
                     "alg_bytes_per_launch": alg,
                     "timing_note": "mean launch = the smaller of two upper bounds from HIP events on the "
                                    "library's stream: an event pair around every tile launch, and the span of "
                                    "the tile launches of steps 2..K over those launches",
                     "alg_bytes_note": "all compressed input words + one index entry per tile per input + dense output"},
    }
    if not args.no_cpu_baseline:
        # the oracle on a prefix of every bitmap: threshold then canonical encoding
        import oracle
        threads = oracle.max_threads()
        cols = np.arange(sample_cols, dtype=np.uint64)
        rs = sample_cols * 64
        t0 = time.perf_counter()
        reps = 0
        while True:
            for t in thetas:
                res = oracle.threshold_cols(host_sample, cols, rs, t)
                oracle.rle_encode(res, rs)
            reps += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": round(reps * q * n * sample_cols * 8 / dt / 1e9, 4), "unit": "GB/s",
                               "cores": threads, "kind": "oracle",
                               "sample": "first %d words of all %d bitmaps (dense, decoding not timed), "
                                         "threshold + canonical encode, %d reps x %d queries, %.1f s"
                                         % (sample_cols, n, reps, q, dt)}
    tq.tq_destroy(ctx)
    return rec


def batch_variant_costs(tq, ctx, table, r, outs, q, avail_rle, stream, copies=16, reps=3):
    """Cost in seconds per query of each variant when the batch path serves it:
    a batch of `copies` copies of the query (distinct outputs) with the
    variant forced, timed with HIP events on the stream around submission
    and completion (median of `reps` after a warm-up), divided by `copies`;
    inf where the variant cannot read the inputs."""
    import numpy as np
    import torch
    bm = tq.bitmap_rows(table, q.members)
    cost = np.full(4, np.inf)
    for v in range(4):
        if v == tq.TQ_VARIANT_RLE and not avail_rle:
            continue
        bq = tq.BatchQueries.from_prepared(
            [tq.PreparedQuery(None, r, outs[k], theta=q.theta, bitmaps=bm, variant=v) for k in range(copies)])
        ts = []
        for rep in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            h = tq.tq_batch_submit(ctx, bq, 0, stream)
            b.record(stream)
            b.synchronize()
            tq.tq_batch_release(h)
            if rep:
                ts.append(a.elapsed_time(b))
        cost[v] = float(np.median(ts)) / 1e3 / copies
    return cost


def train_batch_selector(args, tq, ctx, table, keep_rle, r, outs, pool_n, stream):
    """The selector trained on what the batch path costs: features of seeded
    serving-workload queries (other seeds than the timed ones), their
    per-variant batch costs as targets (log seconds, unavailable variants
    masked), full-batch Adam with the library's kernels; evaluated on
    held-out queries timed the same way."""
    import numpy as np
    import tqgen
    from paper_1402_4073_amd import selector as sel
    ntr, nev = args.serving_train_queries, args.serving_eval_queries
    qs = tqgen.serving_queries(55, count=ntr + nev, pool=pool_n, rate_qps=1.0)
    X = np.zeros((len(qs), 8), dtype=np.float32)
    T = np.zeros((len(qs), 4))
    t0 = time.perf_counter()
    for i, q in enumerate(qs):
        bm = tq.bitmap_rows(table, q.members)
        X[i] = tq.tq_query_features((bm, len(q.members)), r, q.theta)
        T[i] = batch_variant_costs(tq, ctx, table, r, outs, q, bool(keep_rle[list(q.members)].all()), stream)
        if i % 200 == 0:
            print("batch selector data: %d/%d queries, %.0f s" % (i, len(qs), time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
    M = np.isfinite(T).astype(np.float32)
    logT = np.where(np.isfinite(T), np.log(np.where(np.isfinite(T), T, 1.0)), 0.0).astype(np.float32)
    mean, std = sel.normalisation(X[:ntr])
    params, hist = sel.train(ctx, (X[:ntr] - mean) / std, logT[:ntr], M[:ntr], epochs=3000, lr=2e-3)
    lo, hi = X[:ntr].min(axis=0), X[:ntr].max(axis=0)
    pred = sel.predict(ctx, params, (X - mean) / std)
    pred = np.where(M > 0, pred, np.inf)
    te = slice(ntr, len(qs))
    chosen = pred[te].argmin(axis=1)
    Tt = np.where(np.isfinite(T[te]), T[te], np.inf)
    w = {"params": params.tolist(), "mean": mean.tolist(), "std": std.tolist(), "lo": lo.tolist(),
         "hi": hi.tolist(), "margin": 0.0, "queries": len(qs), "train": ntr,
         "context": "batch path (cost per query in a batch of 16 copies)"}
    ev = {"held_out_queries": nev, "regret": sel.regret(Tt, chosen),
          "always_csa_regret": sel.regret(Tt, np.zeros(len(chosen), dtype=int)),
          "best_counts": np.bincount(Tt.argmin(axis=1), minlength=4).tolist(),
          "pick_counts": np.bincount(chosen, minlength=4).tolist(),
          "timing_seconds": round(time.perf_counter() - t0, 1)}
    return w, ev


def bench_serving(args):
    """Serving workload: a pool of 8192 uncompressed bitmaps of r=2^23 bits
    (8 GiB, density log-uniform [1e-4, 0.3]); 20000 queries, each over N
    log-uniform in [2, 1024] distinct pool members with theta uniform in
    [1, N].  Saturation throughput of batched submission (graph replay and
    direct launch) against one tq_threshold call per query, then p50/p99
    latency from arrival to observed completion under Poisson arrivals at
    0.5 / 0.8 / 0.95 of the batched saturation rate, for both."""
    import collections
    import numpy as np
    import torch
    import tqgen
    from paper_1402_4073_amd import binding as tq

    cfg = tqgen.SERVING
    dev = torch.device("cuda:0")
    bs = tqgen.bernoulli_loguniform(6, cfg["pool"], cfg["r_bits"], *cfg["dens"])
    nw, r = bs.nwords, bs.r_bits
    pool = torch.empty((bs.n, nw), dtype=torch.int64, device=dev)
    for j0 in range(0, bs.n, 1024):
        tqgen.fill_gpu(bs, pool[j0:j0 + 1024].reshape(-1), first=j0, count=min(1024, bs.n - j0))
    qs = tqgen.serving_queries(5, count=args.serving_queries, pool=bs.n, rate_qps=1.0)
    nq = len(qs)
    rows = [pool[j] for j in range(bs.n)]
    n_out = 4096
    outs = torch.empty((n_out, nw), dtype=torch.int64, device=dev)
    total_bytes = sum(len(q.members) for q in qs) * nw * 8
    ctx = tq.tq_create(0)
    stream = torch.cuda.Stream(device=dev)
    max_batch = 1024
    slots = max(1, min(4, args.serving_inflight))
    # each batch slot gets its own stream so that small batches overlap (or all share one)
    if args.serving_shared_stream:
        slot_streams = [stream] * slots
    else:
        slot_streams = [torch.cuda.Stream(device=dev) for _ in range(slots)]

    # Registration, before any timing: cardinality and run count of every
    # pool bitmap, and its canonical stream with checkpoint index where that
    # is smaller than the dense words (the hybrid reads each input in its
    # smaller form; the dense words stay registered for every bitmap).
    reg_t0 = time.perf_counter()
    ones_d = torch.zeros(bs.n, dtype=torch.int64, device=dev)
    runs_d = torch.zeros(bs.n, dtype=torch.int64, device=dev)
    with torch.cuda.stream(stream):
        for j in range(bs.n):
            tq.tq_bitmap_stats(ctx, rows[j], r, ones_d[j:j + 1], runs_d[j:j + 1], stream)
        streams, offs, lens, index_pool = tq.encode_pool(ctx, rows, r, stream)
    torch.cuda.synchronize()
    lens_a = np.array(lens, dtype=np.uint64)
    keep_rle = lens_a < nw
    base_s = streams.data_ptr()
    rle_addr = np.where(keep_rle, base_s + 8 * np.array(offs, dtype=np.uint64), 0).astype(np.uint64)
    idx_addr = np.where(keep_rle, index_pool.data_ptr() + np.arange(bs.n, dtype=np.uint64) * index_pool.shape[1] * 8,
                        0).astype(np.uint64)
    table = tq.bitmap_table(np.array([rw.data_ptr() for rw in rows], dtype=np.uint64), rle_addr,
                            np.where(keep_rle, lens_a, 0), idx_addr, ones_d.cpu().numpy().astype(np.uint64),
                            runs_d.cpu().numpy().astype(np.uint64))
    reg_s = time.perf_counter() - reg_t0
    from paper_1402_4073_amd import selector as sel
    batch_weights = os.path.join(ROOT, "paper_1402_4073_amd", "data", "selector_batch_mi355x.json")
    sel_info = {"weights": args.serving_selector}
    if args.serving_selector == "single":
        sel.load_default(ctx)
    elif args.serving_selector == "batch" and os.path.exists(batch_weights):
        sel.load_default(ctx, batch_weights)
        sel_info["weights"] = "batch (shipped)"
    else:
        w, ev = train_batch_selector(args, tq, ctx, table, keep_rle, r, outs, bs.n, stream)
        sel_info["weights"] = "batch (trained in this run)"
        sel_info["evaluation"] = ev
        if args.selector_out:
            os.makedirs(args.selector_out, exist_ok=True)
            with open(os.path.join(args.selector_out, "selector_batch.json"), "w") as fh:
                json.dump(w, fh)
        tq.tq_selector_set(ctx, np.array(w["params"], dtype=np.float32), np.array(w["mean"], dtype=np.float32),
                           np.array(w["std"], dtype=np.float32), np.array(w["lo"], dtype=np.float32),
                           np.array(w["hi"], dtype=np.float32), 0.0)

    # host arrays are marshalled once, outside every timed region: plain
    # pointer arrays for the carry-save-only batches, registered inputs with
    # the selector's choice for the others
    specs_csa = [tq.PreparedQuery([rows[m] for m in q.members], r, outs[i % n_out], theta=q.theta, tag=i)
                 for i, q in enumerate(qs)]
    specs_sel = [tq.PreparedQuery(None, r, outs[i % n_out], theta=q.theta, tag=i,
                                  bitmaps=tq.bitmap_rows(table, q.members), variant=tq.TQ_VARIANT_AUTO)
                 for i, q in enumerate(qs)]
    specs = specs_csa
    chosen = np.zeros(tq.TQ_SEL_VARIANTS, dtype=np.int64)

    def run_batched(arrivals, flags, count_variants=False):
        """Serve queries arriving at `arrivals` (seconds); returns (elapsed, latencies)."""
        inflight = collections.deque()
        done_at = np.zeros(nq)
        nxt = 0
        completed = 0
        t0 = time.perf_counter()
        while completed < nq:
            now = time.perf_counter() - t0
            if nxt < nq and arrivals[nxt] <= now and len(inflight) < slots:
                hi = nxt
                while hi < nq and hi - nxt < max_batch and arrivals[hi] <= now:
                    hi += 1
                bq = tq.BatchQueries.from_prepared(specs[nxt:hi])
                busy = {ent[4] for ent in inflight}
                si = next(k for k in range(slots) if k not in busy)
                h = tq.tq_batch_submit(ctx, bq, flags, slot_streams[si])
                inflight.append([h, nxt, hi, 0, si])
                nxt = hi
                continue
            for ent in list(inflight):
                h, a, b, seen, _ = ent
                d = tq.tq_batch_poll(h)
                if d > seen:
                    t = time.perf_counter() - t0
                    if b - a == 1:
                        done_at[a] = t
                    else:
                        recs = tq.tq_batch_records(h, b - a)
                        newly = (recs["done"] != 0) & (done_at[a:b] == 0.0)
                        done_at[a:b][newly] = t
                    completed += d - seen
                    ent[3] = d
                if ent[3] == b - a:
                    if count_variants:
                        recs = tq.tq_batch_records(h, b - a)
                        chosen[:] += np.bincount(recs["variant"], minlength=tq.TQ_SEL_VARIANTS)[:tq.TQ_SEL_VARIANTS]
                    tq.tq_batch_release(h)
                    inflight.remove(ent)
        elapsed = time.perf_counter() - t0
        lat = [done_at[i] - arrivals[i] for i in range(nq)]
        return elapsed, lat

    def run_single(arrivals):
        """One tq_threshold call per query as it arrives; completion by event."""
        pending = collections.deque()
        done_at = [0.0] * nq
        nxt = 0
        completed = 0
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            while completed < nq:
                now = time.perf_counter() - t0
                while nxt < nq and arrivals[nxt] <= now and len(pending) < 2048:
                    tq.tq_threshold_prepared(ctx, specs[nxt], stream)
                    ev = torch.cuda.Event()
                    ev.record(stream)
                    pending.append((nxt, ev))
                    nxt += 1
                while pending and pending[0][1].query():
                    i, _ = pending.popleft()
                    done_at[i] = time.perf_counter() - t0
                    completed += 1
        elapsed = time.perf_counter() - t0
        return elapsed, [done_at[i] - arrivals[i] for i in range(nq)]

    def pct(v, p):
        return float(np.percentile(np.array(v), p))

    zero = [0.0] * nq
    # warm up every path (graph instantiation, staging caches)
    warm = min(nq, 2000)
    nq_full = nq
    nq = warm
    for sp in (specs_csa, specs_sel):
        specs = sp[:warm]
        run_batched([0.0] * warm, 0)
        run_batched([0.0] * warm, tq.TQ_BATCH_NO_GRAPH)
    specs = specs_csa[:warm]
    run_single([0.0] * warm)
    nq = nq_full
    torch.cuda.synchronize()

    res = {}
    specs = specs_csa
    el_g, _ = run_batched(zero, 0)
    el_d, _ = run_batched(zero, tq.TQ_BATCH_NO_GRAPH)
    el_s, _ = run_single(zero)
    specs = specs_sel
    el_sg, _ = run_batched(zero, 0, count_variants=True)
    el_sd, _ = run_batched(zero, tq.TQ_BATCH_NO_GRAPH)
    specs = specs_csa
    sat_qps = nq / el_g
    # word-column schedule chosen by the autotuner on one full batch, then the
    # saturation run again (the latency runs below keep the default schedule)
    with torch.cuda.stream(stream):
        tuned = tq.tq_batch_tune(ctx, tq.BatchQueries.from_prepared(specs[:max_batch]), stream)
    el_t, _ = run_batched(zero, 0)
    tq.tq_batch_set_schedule(ctx, 4, 16)
    res["saturation"] = {
        "batched_selector_graph": {"qps": round(nq / el_sg, 1), "GBps": round(total_bytes / el_sg / 1e9, 1)},
        "batched_selector_direct": {"qps": round(nq / el_sd, 1), "GBps": round(total_bytes / el_sd / 1e9, 1)},
        "batched_graph": {"qps": round(nq / el_g, 1), "GBps": round(total_bytes / el_g / 1e9, 1)},
        "batched_direct": {"qps": round(nq / el_d, 1), "GBps": round(total_bytes / el_d / 1e9, 1)},
        "per_query_launch": {"qps": round(nq / el_s, 1), "GBps": round(total_bytes / el_s / 1e9, 1)},
        "batched_graph_tuned_schedule": {"qps": round(nq / el_t, 1), "GBps": round(total_bytes / el_t / 1e9, 1),
                                         "items_per_wave": tuned[0], "min_item_work": tuned[1]},
        "default_schedule": {"items_per_wave": 4, "min_item_work": 16},
        "note": "batched_* without 'selector': every query runs the carry-save variant (pointer arrays); "
                "batched_selector_*: registered inputs, variant chosen per query by the shipped selector",
    }
    res["selector_choices"] = {tq.VARIANT_NAMES[v]: int(chosen[v]) for v in range(tq.TQ_SEL_VARIANTS)}
    res["selector"] = sel_info
    res["registration"] = {"seconds": round(reg_s, 2), "compressed_forms": int(keep_rle.sum()),
                           "compressed_words": int(lens_a[keep_rle].sum())}
    res["latency_ms"] = {}
    base_arr = [q.arrival_s for q in qs]      # Poisson with rate 1 query/s
    for frac in (0.5, 0.8, 0.95):
        # the same offered rates for every path: fractions of the carry-save batched saturation
        rate = frac * sat_qps
        arr = [a / rate for a in base_arr]
        specs = specs_sel
        _, lsel = run_batched(arr, 0)
        specs = specs_csa
        _, lb = run_batched(arr, 0)
        _, ld = run_batched(arr, tq.TQ_BATCH_NO_GRAPH)
        _, ls = run_single(arr)
        res["latency_ms"]["%.2f" % frac] = {
            "offered_qps": round(rate, 1),
            "batched_selector": {"p50": round(pct(lsel, 50) * 1e3, 3), "p99": round(pct(lsel, 99) * 1e3, 3)},
            "batched": {"p50": round(pct(lb, 50) * 1e3, 3), "p99": round(pct(lb, 99) * 1e3, 3)},
            "batched_direct": {"p50": round(pct(ld, 50) * 1e3, 3), "p99": round(pct(ld, 99) * 1e3, 3)},
            "per_query_launch": {"p50": round(pct(ls, 50) * 1e3, 3), "p99": round(pct(ls, 99) * 1e3, 3)},
        }
    st = tq.tq_ctx_check(ctx, stream)
    if st != 0:
        raise RuntimeError("device error: %s" % tq.status_string(st))
    tq.tq_destroy(ctx)
    rec = {
        "metric": "batched serving throughput (queries/s) and p50/p99 latency",
        "value": res["saturation"]["batched_selector_graph"]["qps"],
        "unit": "queries/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(el_sg * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64 bitwise", "data": "synthetic (seeded Bernoulli pool resident in HBM)",
        "config": {"workload": "serving: pool 8192 x r=2^23 bits (8 GiB), %d queries, N log-uniform [2,1024], "
                               "theta uniform [1,N], Poisson arrivals; variant per query from the shipped "
                               "selector over registered inputs" % nq,
                   "logical_input_bytes": total_bytes, "max_batch": max_batch, "slots": slots,
                   "shared_stream": bool(args.serving_shared_stream)},
        "serving": res,
    }
    return rec


def bench_selector(args):
    """Selector workload: queries with N log-uniform in [2, 4096], r = 2^22,
    density log-uniform in [1e-5, 0.5], mean ones-run log-uniform in
    [1, 4096], theta/N uniform in (0, 1].  Every query's bitmaps are
    generated on the GPU and registered in both forms (dense words; canonical
    stream with checkpoint index; cardinality and run count), the four
    variants are timed (median of 5 after a warm-up), the network is trained
    on the first queries' log times with the library's kernels and evaluated
    on the rest: regret against the exhaustive best, with and without the
    exhaustive-timing fallback, against always running the default variant."""
    import numpy as np
    import torch
    import tqgen
    from paper_1402_4073_amd import binding as tq
    from paper_1402_4073_amd import selector as sel

    if args.selector_out:
        os.makedirs(args.selector_out, exist_ok=True)
    r = tqgen.SELECTOR["r_bits"]
    nw = (r + 63) // 64
    qs = tqgen.selector_queries(4, count=args.selector_queries)
    ctx = tq.tq_create(0)
    dev = torch.device("cuda:0")
    nq = len(qs)
    X = np.zeros((nq, 8), dtype=np.float32)
    Tm = np.zeros((nq, 4), dtype=np.float64)      # median seconds per variant
    meta = []
    iw = tq.tq_rle_index_words(r)
    t_start = time.perf_counter()
    for qi, q in enumerate(qs):
        ms = tqgen.markov_density_runlength(q.seed, q.n, r, q.density, q.mean_run)
        dense = torch.empty((q.n, nw), dtype=torch.int64, device=dev)
        tqgen.fill_gpu(ms, dense.view(-1))
        slots = torch.empty((q.n, nw + 2), dtype=torch.int64, device=dev)
        idx = torch.empty((q.n, iw), dtype=torch.int64, device=dev)
        lens = torch.zeros(q.n, dtype=torch.int64, device=dev)
        stats = torch.zeros((q.n, 2), dtype=torch.int64, device=dev)
        for j in range(q.n):
            tq.tq_bitmap_stats(ctx, dense[j], r, stats[j, 0:1], stats[j, 1:2])
            tq.tq_rle_encode(ctx, dense[j], r, slots[j], nw + 2, lens[j:j + 1], idx[j])
        if tq.tq_ctx_check(ctx) != 0:
            raise RuntimeError("encode failed")
        st = stats.cpu().numpy()
        ln = lens.cpu().numpy()
        bms = [dict(dense=dense[j], rle=(slots[j], int(ln[j]), idx[j]), ones=int(st[j, 0]), runs=int(st[j, 1]))
               for j in range(q.n)]
        arr = (tq.bitmap_array(bms), q.n)
        X[qi] = tq.tq_query_features(arr, r, q.theta)
        out = torch.empty(nw, dtype=torch.int64, device=dev)
        for v in range(4):
            tq.tq_threshold_variant(ctx, arr, r, q.theta, v, out)      # warm-up
            evs = []
            for _ in range(5):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                tq.tq_threshold_variant(ctx, arr, r, q.theta, v, out)
                b.record()
                evs.append((a, b))
            torch.cuda.synchronize()
            Tm[qi, v] = float(np.median([a.elapsed_time(b) for a, b in evs])) / 1e3
        meta.append(dict(n=q.n, theta=q.theta, density=q.density, mean_run=q.mean_run,
                         comp_words=int(ln.sum())))
        del dense, slots, idx
        if qi % 250 == 0:
            print("selector data: %d/%d queries, %.0f s" % (qi, nq, time.perf_counter() - t_start),
                  file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    ntr = min(args.selector_train, nq - 1)
    logT = np.log(Tm)
    mean, std = sel.normalisation(X[:ntr])
    Xn = (X - mean) / std
    t0 = time.perf_counter()
    params, hist = sel.train(ctx, Xn[:ntr], logT[:ntr].astype(np.float32), epochs=4000, lr=2e-3)
    train_s = time.perf_counter() - t0
    pred = sel.predict(ctx, params, Xn)
    te = slice(ntr, nq)
    P, Ttest = pred[te], Tm[te]
    chosen = P.argmin(axis=1)
    best_t = Ttest.min(axis=1)
    res = {"selector": sel.regret(Ttest, chosen)}
    res["always_csa"] = sel.regret(Ttest, np.zeros(len(chosen), dtype=int))
    fixed = int(np.argmin(Tm[:ntr].sum(axis=0)))
    res["best_fixed_variant"] = dict(sel.regret(Ttest, np.full(len(chosen), fixed)), variant=tq.VARIANT_NAMES[fixed])
    # fallback: when the top two predictions are within the margin or the
    # features leave the training range, time all variants (their cost counts)
    srt = np.sort(P, axis=1)
    margin = 0.0
    lo, hi = X[:ntr].min(axis=0), X[:ntr].max(axis=0)
    out_of_range = ~np.all((X[te] >= lo) & (X[te] <= hi), axis=1)
    unsure = ((srt[:, 1] - srt[:, 0]) < margin) | out_of_range
    eff = np.where(unsure, Ttest.sum(axis=1), Ttest[np.arange(len(chosen)), chosen])
    res["selector_with_fallback"] = {"workload": float(eff.sum() / best_t.sum() - 1.0),
                                     "fallback_rate": float(unsure.mean()), "margin": margin}
    wins = np.bincount(Ttest.argmin(axis=1), minlength=4)
    picks = np.bincount(chosen, minlength=4)
    res["best_variant_counts"] = {tq.VARIANT_NAMES[v]: int(wins[v]) for v in range(4)}
    res["selector_pick_counts"] = {tq.VARIANT_NAMES[v]: int(picks[v]) for v in range(4)}
    res["speedup_vs_always_csa"] = float(Ttest[:, 0].sum() / Ttest[np.arange(len(chosen)), chosen].sum())
    res["train"] = {"queries": ntr, "epochs": 4000, "seconds": round(train_s, 2), "loss_first_last": [hist[0][1], hist[-1][1]]}
    # held-out queries through the library's own dispatch (host inference)
    tq.tq_selector_set(ctx, params, mean, std, lo, hi, margin)
    agree = sum(int(np.argmin(tq.tq_selector_predict(ctx, X[i]))) == int(pred[i].argmin()) for i in range(ntr, nq))
    res["host_gpu_inference_agreement"] = agree / (nq - ntr)
    if args.selector_out:
        np.savez(os.path.join(args.selector_out, "dataset.npz"), X=X, T=Tm, params=params, mean=mean, std=std)
        with open(os.path.join(args.selector_out, "weights.json"), "w") as fh:
            json.dump({"params": params.tolist(), "mean": mean.tolist(), "std": std.tolist(), "lo": lo.tolist(),
                       "hi": hi.tolist(), "margin": margin, "queries": nq, "train": ntr,
                       "features": ["log2 N", "theta/N", "log10 density", "log10 ones-run", "std log10 density",
                                    "log2 r", "log2 compression", "log2 theta/(1+E count)"],
                       "variants": list(tq.VARIANT_NAMES)}, fh)
    tq.tq_destroy(ctx)
    return {
        "metric": "selector regret on held-out queries (sum t_selected / sum t_best - 1)",
        "value": round(res["selector"]["workload"], 4), "unit": "fraction", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round((time.perf_counter() - t_start) * 1e3, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "fp32 (selection only)",
        "data": "synthetic (seeded Markov bitmaps generated per query)",
        "config": {"workload": "selector: %d queries (%d train / %d held out), r=2^22, N log-uniform [2,4096], "
                               "density log-uniform [1e-5,0.5], mean ones-run log-uniform [1,4096]"
                               % (nq, ntr, nq - ntr)},
        "results": res,
    }


def selector_summary(args, held_out=range(2000, 2048)):
    """The shipped selector on queries of the selector workload held out from
    its training: every variant timed, the
    library's own dispatch (tq_threshold_auto, no timing fallback) asked for
    its choice; regret against the exhaustive best and gain over always
    running the carry-save variant (timings: median of 5 after a warm-up)."""
    import numpy as np
    import torch
    import tqgen
    from paper_1402_4073_amd import binding as tq
    from paper_1402_4073_amd import selector as sel
    ctx = tq.tq_create(0)
    sel.load_default(ctx)
    r = tqgen.SELECTOR["r_bits"]
    nw = (r + 63) // 64
    iw = tq.tq_rle_index_words(r)
    qs = tqgen.selector_queries(4, count=held_out.stop)
    dev = torch.device("cuda:0")
    T = np.zeros((len(held_out), 4))
    chosen = np.zeros(len(held_out), dtype=int)
    t0 = time.perf_counter()
    for k, qi in enumerate(held_out):
        q = qs[qi]
        ms = tqgen.markov_density_runlength(q.seed, q.n, r, q.density, q.mean_run)
        dense = torch.empty((q.n, nw), dtype=torch.int64, device=dev)
        tqgen.fill_gpu(ms, dense.view(-1))
        slots = torch.empty((q.n, nw + 2), dtype=torch.int64, device=dev)
        idx = torch.empty((q.n, iw), dtype=torch.int64, device=dev)
        lens = torch.zeros(q.n, dtype=torch.int64, device=dev)
        stats = torch.zeros((q.n, 2), dtype=torch.int64, device=dev)
        for j in range(q.n):
            tq.tq_bitmap_stats(ctx, dense[j], r, stats[j, 0:1], stats[j, 1:2])
            tq.tq_rle_encode(ctx, dense[j], r, slots[j], nw + 2, lens[j:j + 1], idx[j])
        st, ln = stats.cpu().numpy(), lens.cpu().numpy()
        arr = (tq.bitmap_array([dict(dense=dense[j], rle=(slots[j], int(ln[j]), idx[j]), ones=int(st[j, 0]),
                                     runs=int(st[j, 1])) for j in range(q.n)]), q.n)
        out = torch.empty(nw, dtype=torch.int64, device=dev)
        for v in range(4):
            tq.tq_threshold_variant(ctx, arr, r, q.theta, v, out)
            evs = []
            for _ in range(5):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                tq.tq_threshold_variant(ctx, arr, r, q.theta, v, out)
                b.record()
                evs.append((a, b))
            torch.cuda.synchronize()
            T[k, v] = float(np.median([a.elapsed_time(b) for a, b in evs])) / 1e3
        chosen[k] = tq.tq_threshold_auto(ctx, arr, r, q.theta, out, 0)
        del dense, slots, idx
    if tq.tq_ctx_check(ctx) != 0:
        raise RuntimeError("device error in the selector summary")
    tq.tq_destroy(ctx)
    torch.cuda.empty_cache()
    reg = sel.regret(T, chosen)
    return {"queries": len(held_out), "held_out_of": "selector workload (r=2^22, seeded), queries %d-%d"
            % (held_out.start, held_out.stop - 1),
            "regret": round(reg["workload"], 4), "per_query_regret": round(reg["per_query_mean"], 4),
            "gain_over_always_csa": round(float(T[:, 0].sum() / T[np.arange(len(chosen)), chosen].sum()), 3),
            "picks": np.bincount(chosen, minlength=4).tolist(), "best": np.bincount(T.argmin(axis=1), minlength=4).tolist(),
            "seconds": round(time.perf_counter() - t0, 1)}


SELECTOR_IDLE_S = 20


def summaries(args):
    """Compact figures of the RLE, serving and selector workloads for the
    default run (each also has a full run of its own: --workload ...)."""
    import copy
    import torch
    out = {}
    a = copy.copy(args)
    a.steps, a.warmup, a.no_cpu_baseline = 3, 1, True
    r = bench_rle(a)
    out["rle"] = {"metric": r["metric"], "value": r["value"], "unit": r["unit"],
                  "per_query_ms": r["per_query_ms"], "tile_kernel_ms": r["tile_kernel_ms"],
                  "no_index_dense_query_ms": r["no_index_dense_query_ms"],
                  "compressed_input_GBps": r["compressed_input_GBps"],
                  "roofline": {k: r["roofline"][k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")}}
    torch.cuda.empty_cache()
    a = copy.copy(args)
    a.serving_selector = "batch"
    sv = bench_serving(a)["serving"]
    out["serving"] = {"unit": "queries/s", "saturation": {k: v["qps"] for k, v in sv["saturation"].items()
                                                          if isinstance(v, dict) and "qps" in v},
                      "latency_ms_at_0.8": sv["latency_ms"]["0.80"], "selector_choices": sv["selector_choices"]}
    torch.cuda.empty_cache()
    # The selector's weights come from timings taken at steady clocks.  Right
    # after a sustained load the clock is lower for a while, which slows the
    # vector-ALU-bound variants (the per-position counter) more than the
    # memory-bound ones and so moves the exhaustive best: the regret is taken
    # both right after the serving run and after an idle of SELECTOR_IDLE_S,
    # and the latter is the figure reported as the selector's.
    hot = selector_summary(args)
    time.sleep(SELECTOR_IDLE_S)
    out["selector"] = selector_summary(args)
    out["selector"]["idle_before_s"] = SELECTOR_IDLE_S
    out["selector"]["right_after_serving"] = {k: hot[k] for k in ("regret", "per_query_regret",
                                                                   "gain_over_always_csa", "picks", "best")}
    return out


def time_graph_step(torch, one_step, stream, steps):
    """The step's queries captured once into a HIP graph (every array they
    stage was staged by the eager passes on the same stream) and replayed:
    launch-bound small queries lose most of their per-call host cost."""
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=stream):
        one_step(None)
    g.replay()
    torch.cuda.synchronize()
    reps = max(steps, 20)
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"ms_per_step": round(dt / reps * 1e3, 4), "steps": reps,
            "note": "the same queries captured into one graph and replayed (wall time per replay)"}


def time_consumers(tq, ctx, rows, r, nw, stream, steps):
    """Fused consumers of a result (threshold 16): the plain query, the query
    with an AND filter and a count in the same pass, and the count alone."""
    import torch
    theta = 16
    out = torch.empty(nw, dtype=torch.int64, device=rows[0].device)
    cnt = torch.zeros(1, dtype=torch.int64, device=rows[0].device)
    filt = rows[1]
    runs = {
        "threshold_ms": lambda: tq.tq_threshold(ctx, rows, r, theta, out, stream),
        "threshold_and_filter_and_count_ms": lambda: tq.tq_threshold_fused(ctx, rows, r, theta, filt, out, cnt,
                                                                           stream),
        "count_only_ms": lambda: tq.tq_threshold_fused(ctx, rows, r, theta, None, None, cnt, stream),
    }
    res = {"theta": theta}
    with torch.cuda.stream(stream):
        for name, fn in runs.items():
            fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            res[name] = round(e0.elapsed_time(e1) / steps, 4)
    if tq.tq_ctx_check(ctx, stream) != 0:
        raise RuntimeError("device error in the consumer timings")
    return res


def time_weighted(tq, ctx, rows, r, nw, stream, steps):
    """Weighted threshold with weights 1..4 (cycling over the inputs), theta =
    half the total: one read of each input, against the same query through
    replication (input j listed w_j times, section 2.3)."""
    import torch
    weights = [1 + (j % 4) for j in range(len(rows))]
    theta = sum(weights) // 2
    rep = [rows[j] for j in range(len(rows)) for _ in range(weights[j])]
    out = torch.empty(nw, dtype=torch.int64, device=rows[0].device)
    runs = {
        "weighted_ms": lambda: tq.tq_threshold_weighted(ctx, rows, weights, r, theta, out, stream),
        "replicated_ms": lambda: tq.tq_threshold(ctx, rep, r, theta, out, stream),
    }
    res = {"weights": "1 + (j mod 4)", "theta": theta, "total_weight": sum(weights)}
    with torch.cuda.stream(stream):
        for name, fn in runs.items():
            fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            res[name] = round(e0.elapsed_time(e1) / steps, 4)
    if tq.tq_ctx_check(ctx, stream) != 0:
        raise RuntimeError("device error in the weighted timings")
    return res


def time_autotune(tq, tqgen, r_large, rows_large, stream, steps):
    """Threshold queries under the default launch-shape rule and under the
    autotuner's choice (tuned on the first query of the class), for the large
    workload and two other shapes: few inputs, and many inputs over short
    bitmaps."""
    import torch
    dev = rows_large[0].device
    shapes = [("N=256 r=2^26", rows_large, r_large, 16)]
    small = tqgen.bernoulli_fixed(1, 16, 1 << 20, 0.05)
    p_small = torch.empty((small.n, small.nwords), dtype=torch.int64, device=dev)
    tqgen.fill_gpu(small, p_small.view(-1))
    shapes.append(("N=16 r=2^20", [p_small[j] for j in range(small.n)], small.r_bits, 2))
    wide = tqgen.bernoulli_fixed(3, 4096, 1 << 18, 0.05)
    p_wide = torch.empty((wide.n, wide.nwords), dtype=torch.int64, device=dev)
    tqgen.fill_gpu(wide, p_wide.view(-1))
    shapes.append(("N=4096 r=2^18", [p_wide[j] for j in range(wide.n)], wide.r_bits, 200))
    res = {}
    for name, rows, r, theta in shapes:
        nw = (r + 63) // 64
        out = torch.empty(nw, dtype=torch.int64, device=dev)
        ptrs = tq.ptr_array(rows)
        ctx = tq.tq_create(0)
        ent = {"theta": theta}
        # the launch shapes of the single counter kernel (inputs not split
        # over workgroups: time_split covers that)
        tq.tq_set_option(ctx, tq.TQ_OPTION_SPLIT, 0)
        tq.tq_set_option(ctx, tq.TQ_OPTION_AUTOTUNE, 1)
        with torch.cuda.stream(stream):
            tq.raw_threshold(ctx, ptrs, len(rows), r, theta, out.data_ptr(), stream)   # tunes the class
            torch.cuda.synchronize()
        # enough launches for a stable mean on short queries; the two settings
        # alternate so that clock drift affects both alike
        reps = max(steps, int(2e-3 / max(1e-6, r * len(rows) / 8 / 6e12)))
        reps = min(reps, 2000)
        acc = {"default_ms": 0.0, "tuned_ms": 0.0}
        for _ in range(3):
            for label, auto in (("default_ms", 0), ("tuned_ms", 1)):
                tq.tq_set_option(ctx, tq.TQ_OPTION_AUTOTUNE, auto)
                with torch.cuda.stream(stream):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(reps):
                        tq.raw_threshold(ctx, ptrs, len(rows), r, theta, out.data_ptr(), stream)
                    e1.record(stream)
                    torch.cuda.synchronize()
                acc[label] += e0.elapsed_time(e1) / reps / 3
        ent.update({k: round(v, 4) for k, v in acc.items()})
        ent["launches"] = 3 * reps
        lines = tq.tq_tune_export(ctx).strip().splitlines()
        ent["tuned_shape"] = lines[0].split(":")[1].strip() if lines else None
        if tq.tq_ctx_check(ctx, stream) != 0:
            raise RuntimeError("device error in the autotune timings")
        tq.tq_destroy(ctx)
        res[name] = ent
    res["shape_fields"] = "words per lane, waves splitting the inputs, column groups per workgroup, 0"
    return res


def time_split(tq, tqgen, dev, stream, steps):
    """Short bitmaps with many inputs: the inputs split over workgroups (two
    kernels, partial counts added by the second) against one counter kernel
    with at most eight waves per column group, same queries."""
    import torch
    res = {}
    for name, n, r, theta in (("N=5000 r=200 words", 5000, 200 * 64, 1500), ("N=4096 r=2^18", 4096, 1 << 18, 200)):
        bs = tqgen.bernoulli_loguniform(12, n, r, 1e-4, 0.5)
        pool = torch.empty((n, bs.nwords), dtype=torch.int64, device=dev)
        tqgen.fill_gpu(bs, pool.view(-1))
        rows = [pool[j] for j in range(n)]
        out = torch.empty(bs.nwords, dtype=torch.int64, device=dev)
        ptrs = tq.ptr_array(rows)
        ctx = tq.tq_create(0)
        reps = max(steps, 200)
        acc = {"split_us": 0.0, "single_kernel_us": 0.0}
        with torch.cuda.stream(stream):
            for _ in range(3):
                for label, on in (("split_us", 1), ("single_kernel_us", 0)):
                    tq.tq_set_option(ctx, tq.TQ_OPTION_SPLIT, on)
                    tq.raw_threshold(ctx, ptrs, n, r, theta, out.data_ptr(), stream)
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(reps):
                        tq.raw_threshold(ctx, ptrs, n, r, theta, out.data_ptr(), stream)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    acc[label] += e0.elapsed_time(e1) * 1e3 / reps / 3
        if tq.tq_ctx_check(ctx, stream) != 0:
            raise RuntimeError("device error in the split timings")
        tq.tq_destroy(ctx)
        in_bytes = n * bs.nwords * 8
        res[name] = {"theta": theta, "input_bytes": in_bytes, **{k: round(v, 2) for k, v in acc.items()},
                     "split_GBps": round(in_bytes / acc["split_us"] / 1e3, 1),
                     "single_kernel_GBps": round(in_bytes / acc["single_kernel_us"] / 1e3, 1)}
        del pool, rows
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.record_traffic:
        record_traffic(args.record_traffic)
        return
    if args.copy_calibration:
        copy_calibration()
        return

    if args.workload == "rle":
        print(json.dumps(bench_rle(args)), flush=True)
        return
    if args.workload == "serving":
        print(json.dumps(bench_serving(args)), flush=True)
        return
    if args.workload == "selector":
        print(json.dumps(bench_selector(args)), flush=True)
        return

    import numpy as np
    import torch
    import tqgen
    from paper_1402_4073_amd import binding as tq

    dev = torch.device("cuda:0")
    if args.workload == "large":
        bs = tqgen.large_set(2)
        thetas = tqgen.LARGE["thetas"]
        lo, hi = tqgen.LARGE["interval"]
        desc = ("large uncompressed: N=256 bitmaps, r=2^26 bits, density log-uniform "
                "[1e-4,0.5]; thresholds 2,16,128,255 + interval 2..10 + parity")
    else:
        bs = tqgen.small_set(1)
        thetas = tqgen.SMALL["thetas"]
        lo, hi = 2, 10
        desc = "small: N=16 bitmaps, r=2^20 bits, Bernoulli(0.05); thresholds 1,2,8,16 + interval + parity"
    n, nw, r = bs.n, bs.nwords, bs.r_bits
    pool = torch.empty((n, nw), dtype=torch.int64, device=dev)
    tqgen.fill_gpu(bs, pool.view(-1))
    rows = [pool[j] for j in range(n)]
    out = torch.empty(nw, dtype=torch.int64, device=dev)
    queries = [("threshold", t) for t in thetas]
    queries += [("symmetric", tq.truth_interval(n, lo, hi)), ("symmetric", tq.truth_parity(n))]

    ctx = tq.tq_create(0)
    stream = torch.cuda.Stream(device=dev)
    # registration, before any timing: each bitmap's cardinality (and run
    # count), by which threshold queries order their inputs
    stats = torch.zeros((n, 2), dtype=torch.int64, device=dev)
    for j in range(n):
        tq.tq_bitmap_stats(ctx, rows[j], r, stats[j, 0:1], stats[j, 1:2])
    st_host = stats.cpu().numpy()
    registered = (tq.bitmap_array([dict(dense=rows[j], rle=None, ones=int(st_host[j, 0]), runs=int(st_host[j, 1]))
                                   for j in range(n)]), n)

    def one_step(events):
        for kind, arg in queries:
            if events is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            if kind == "threshold":
                tq.tq_threshold_variant(ctx, registered, r, arg, tq.TQ_VARIANT_CSA, out, stream)
            else:
                tq.tq_symmetric(ctx, rows, r, arg, out, stream)
            if events is not None:
                e1.record(stream)
                events.append((e0, e1))

    def timed_pass(prune):
        # the roofline pass (prune 0) runs every query on the carry-save kernel
        tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, prune)
        tq.tq_set_option(ctx, tq.TQ_OPTION_LOOPED, prune)
        events = []
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                one_step(None)
            torch.cuda.synchronize()
            if tq.tq_ctx_check(ctx, stream) != 0:
                raise RuntimeError("device error during warmup")
            # r0 / r1 bracket the launches of steps 2..K: recorded once the
            # first step is queued, so the device is never idle between them
            r0 = torch.cuda.Event(enable_timing=True)
            r1 = torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            for s in range(args.steps):
                if s == 1:
                    r0.record(stream)
                one_step(events)
            r1.record(stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        st = tq.tq_ctx_check(ctx, stream)
        if st != 0:
            raise RuntimeError("device error: %s" % tq.status_string(st))
        region = (r0.elapsed_time(r1), (args.steps - 1) * len(queries)) if args.steps > 1 else None
        return t1 - t0, [a.elapsed_time(b) for a, b in events], region

    # the reported throughput: the library as configured (threshold pruning on by default)
    elapsed, query_ms, _ = timed_pass(args.prune)
    # the roofline: every input word read (no pruning), so algorithmic bytes are the bytes moved
    _, kernel_ms, region = timed_pass(0)
    tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, 1)
    tq.tq_set_option(ctx, tq.TQ_OPTION_LOOPED, 1)
    graph = time_graph_step(torch, one_step, stream, args.steps) if args.workload == "small" else None
    consumers = None if args.no_consumers else time_consumers(tq, ctx, rows, r, nw, stream, args.steps)
    weighted = None if args.no_consumers else time_weighted(tq, ctx, rows, r, nw, stream, args.steps)
    autotune = None
    split = None
    if args.workload == "large" and not args.no_consumers:
        autotune = time_autotune(tq, tqgen, r, rows, stream, args.steps)
        split = time_split(tq, tqgen, dev, stream, args.steps)
    # average launch, bounded from above twice: by an event pair around every
    # launch (each pair adds its own overhead) and by the span of steps 2..K
    # over their launches (the span also holds the gaps between launches and
    # any other work of the calls); the smaller bound is reported
    mean_event_pair_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    mean_region_s = region[0] / region[1] / 1e3 if region else mean_event_pair_s
    mean_kernel_s = min(mean_event_pair_s, mean_region_s)
    in_bytes_query = n * nw * 8
    out_bytes_query = nw * 8
    alg_bytes = in_bytes_query + out_bytes_query
    achieved = alg_bytes / mean_kernel_s / 1e9
    value = len(queries) * in_bytes_query * args.steps / elapsed / 1e9
    kernel_key = "dense_kernel<K=%d>/%s" % (max(4, n.bit_length()), args.workload)
    traffic = load_traffic(kernel_key)

    rec = {
        "metric": "input GB/s per threshold query (logical input bytes / wall time)",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 bitwise",
        "data": "synthetic (seeded counter-based generator, resident in HBM)",
        "config": {"workload": desc, "n_bitmaps": n, "r_bits": r, "queries_per_step": len(queries),
                   "input_bytes_per_query": in_bytes_query},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kernel_key, "mean_launch_us": round(mean_kernel_s * 1e6, 2),
                     "mean_launch_us_event_pair_each": round(mean_event_pair_s * 1e6, 2),
                     "mean_launch_us_span": round(mean_region_s * 1e6, 2),
                     "alg_bytes_per_launch": alg_bytes,
                     "note": "launches with pruning off (every input word read); mean launch = the smaller of "
                             "two upper bounds from HIP events on the library's stream: an event pair around "
                             "every launch, and the span of steps 2..K over their launches"},
        "per_query_ms": [round(sum(query_ms[i::len(queries)]) / args.steps, 4) for i in range(len(queries))],
        "per_query_ms_unpruned": [round(sum(kernel_ms[i::len(queries)]) / args.steps, 4)
                                  for i in range(len(queries))],
        "prune": bool(args.prune),
        "input_order": "threshold queries read registered inputs by cardinality (densest first below half "
                       "the mean count, else sparsest first); registration is untimed",
        "consumers": consumers,
        "weighted": weighted,
        "autotune": autotune,
        "split_inputs": split,
    }
    # HBM bytes the timed (pruned) step moves, per query from rocprofv3
    # counters on the same sources and data, over the measured step time
    step_bytes = load_traffic("dense_step/large-pruned", "bytes_per_query") \
        if args.workload == "large" and args.prune else None
    if step_bytes:
        step_s = elapsed / args.steps
        ach = sum(step_bytes) / step_s / 1e9
        rec["pruned_step"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(ach / HBM_PEAK_GBS, 4), "traffic_bytes_per_step": sum(step_bytes),
                              "traffic_bytes_per_query": step_bytes,
                              "note": "bytes the six queries of the timed step move (FETCH_SIZE + WRITE_SIZE "
                                      "per dispatch, scaled by a plain copy) over ms_per_step; the logical "
                                      "`value` counts every input word of every query"}
    if graph:
        rec["graph_replay"] = graph
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(rows, n, nw, r, queries, args.cpu_seconds)
        # one thread, as the paper's single-threaded Java measurements
        rec["cpu_single_thread"] = cpu_baseline(rows, n, nw, r, queries, args.cpu_seconds / 3, threads=1)
    tq.tq_destroy(ctx)
    if args.workload == "large" and not args.no_summaries:
        del pool, rows, out
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        print("summaries of the other workloads ...", file=sys.stderr, flush=True)
        rec["other_workloads"] = summaries(args)
        rec["other_workloads"]["seconds"] = round(time.perf_counter() - t0, 1)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
