#!/usr/bin/env python
"""Benchmark of RotorMap's hot path on one MI355X.

One step = one pass of the whole path over the batch: build the window index
of the reference (rolling encoder), encode every read head, score every read
against every window on MFMA with the fused top-k, merge, and rescore the
candidates in FP32.  Inputs are resident in HBM before timing starts.

Prints ONE JSON line (rank 0).  Default workload: the precision workload
(10 Mbp synthetic reference with 41% GC and 5% repeats, 100,000 reads of
150 bp at 2% error, every stride-1 window, top-8 from 16 candidates
rescored in FP32, FP16 embeddings).
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

METRIC = ("reads mapped/sec at ≥99% top-k recall vs FP64 oracle; window scores/sec")
PEAK_TFLOPS = {"fp32": 157.3, "fp16": 2500.0, "fp8": 5000.0}   # dense MFMA, MI355X
FLOPS_PER_SCORE = 1024  # two 256-long real dot products (Re and Im rows), 2 flops each
HBM_PEAK_GBS = 8000.0


SCORE_SOURCES = (
    "paper_2603_22245_amd/csrc/rm_score.hip",
    "paper_2603_22245_amd/csrc/rm_score_f16.hip",
    "paper_2603_22245_amd/csrc/rm_score_kernel.h",
    "paper_2603_22245_amd/csrc/rm_internal.h",
    "paper_2603_22245_amd/build.py",
)


# sources of the 1,024-component product (K = 2,048)
WIDE_SOURCES = (
    "paper_2603_22245_amd/csrc/rm_wide.hip",
    "paper_2603_22245_amd/csrc/rm_tokens.h",
    "paper_2603_22245_amd/csrc/rm_internal.h",
    "paper_2603_22245_amd/build.py",
)


def score_source_digest(sources=SCORE_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, precision: str, tokens=None, row_reals=None):
    """HBM bytes per scoring launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE of a rocprofv3 --pmc run of this benchmark on
    this workload, scaled by a plain copy's readings), or None when there is no
    summary for this workload, precision and encoding, the summary was taken
    with another row length (row_reals, when given: 256, or 192 for the
    letter-sum form), or the kernel sources changed since it was taken.
    tokens: None (letters, score_topk_kernel) or the name of a 1,024-component
    token encoding (score_wide_kernel)."""
    if tokens is None:
        name, sources = f"score_topk_{precision}_{workload}_traffic.txt", SCORE_SOURCES
    else:
        name, sources = f"score_wide_{precision}_{tokens}_{workload}_traffic.txt", WIDE_SOURCES
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.loads(fh.read().split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None
    if d.get("source_sha256") != score_source_digest(sources):
        return None
    if row_reals is not None and d.get("row_reals", 256) != row_reals:
        return None
    return d.get("bytes_per_launch")


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="precision")
    ap.add_argument("--precision", default=None, help="fp32 | fp16 | fp8 (default: the workload's)")
    ap.add_argument("--reads", type=int, default=None, help="use only the first R reads")
    ap.add_argument("--k-fetch", type=int, default=16)
    ap.add_argument("--coarse-stride", type=int, default=None,
                    help="index at this window stride, then step-1 refinement around the "
                         "candidates (§3.4) in place of the rescore")
    ap.add_argument("--radius", type=int, default=None,
                    help="refinement radius in letters (default: coarse stride - 1)")
    ap.add_argument("--corr-pairs", type=int, default=100_000,
                    help="correlation workload: pairs over all mutation rates")
    ap.add_argument("--tokens", default=None,
                    help="token encoding (s-mers, compact maps): s2 | s3 | s8c16 | s4m4 | "
                         "s8c256 | s4f128 (default: the letter encoding)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the plain FP32 comparison step")
    ap.add_argument("--letter-sum", choices=("auto", "on", "off"), default="auto",
                    help="row form of the headline index: the library's choice (the "
                         "letter-sum form for FP16 letter indexes), or forced on / off")
    ap.add_argument("--no-fp32-letter-sum", action="store_true",
                    help="skip the FP32 leg in the letter-sum form")
    ap.add_argument("--no-fp8-letter-sum", action="store_true",
                    help="skip the FP8 leg in the letter-sum form")
    ap.add_argument("--no-fp8", action="store_true",
                    help="skip the FP8 leg of an FP16 run (default workload)")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the batched leg of the default run")
    ap.add_argument("--no-threshold", action="store_true",
                    help="skip the threshold-regime leg of the default run")
    ap.add_argument("--threshold-floor", type=float, default=0.1,
                    help="second run of the threshold regime with this fidelity floor "
                         "(the first has none)")
    ap.add_argument("--threshold-err", type=float, default=0.02,
                    help="threshold regime: target mutation rate of the per-window thresholds")
    ap.add_argument("--cpu-reads", type=int, default=None,
                    help="oracle baseline: read heads timed (default: 2,000 for the precision "
                         "workload, 1,000 for scale)")
    ap.add_argument("--cpu-windows", type=int, default=262_144)
    ap.add_argument("--pairs", type=int, default=1_000_000, help="learned workload: string pairs")
    ap.add_argument("--epochs", type=int, default=3, help="learned workload: training epochs")
    ap.add_argument("--no-map-rerun", action="store_true",
                    help="learned workload: skip the precision-workload rerun")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration)")
    return ap.parse_args()


def calibrate_copy():
    """A plain copy of known size: 1 GiB read + 1 GiB written, three times."""
    import torch
    n = 1 << 30
    x = torch.ones(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 3}))


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: it measures one GPU's share of the work; "
              "sharding the path across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2603_22245_amd import mapper, _lib as L

    if args.calibrate_copy:
        calibrate_copy()
        return

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.workload == "batching":
        out = bench_batching(args)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "learned":
        out = bench_learned(args)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "correlation":
        out = bench_correlation(args)
        print(json.dumps(out), flush=True)
        return
    w = synth.WORKLOADS[args.workload]
    precision = args.precision or w.precision
    k, k_fetch = w.k, max(w.k, args.k_fetch)

    t0 = time.time()
    ref = w.reference()
    reads = w.reads(ref)
    if args.reads is not None and args.reads < reads.n:
        n = args.reads
        reads = synth.Reads(reads.seq[:reads.offsets[n]], reads.offsets[:n + 1], reads.truth[:n])
    R = reads.n
    log(f"workload {w.name}: G={ref.shape[0]:,} R={R:,} generated in {time.time() - t0:.1f}s")

    coarse = args.coarse_stride is not None and args.coarse_stride > 1
    stride = args.coarse_stride if coarse else w.stride
    radius = (args.radius if args.radius is not None else stride - 1) if coarse else 0
    tok = {}
    token_map_ms = None
    if args.tokens is not None:
        s_, m_, c_, tm_, sched_ = synth.token_encoding(args.tokens)
        if synth.token_map_is_frequent(args.tokens):  # the reference's most frequent s-mers
            t_map = time.perf_counter()
            tm_, _ = mapper.frequent_token_map(ref, s_, c_)
            torch.cuda.synchronize()
            token_map_ms = (time.perf_counter() - t_map) * 1e3
        tok = dict(mer_len=s_, n_freq=m_, n_class=c_, token_map=tm_, schedule=sched_)
        if c_ * m_ != 128 and precision == "fp32":
            print("encodings of 1,024 components have FP16 and FP8 indexes only", file=sys.stderr)
            sys.exit(2)
    wide = bool(tok) and tok["n_class"] * tok["n_freq"] != 128

    run = run_map(args, w, ref, reads, precision, k, k_fetch, stride, radius, tok,
                  args.steps, args.warmup,
                  reduced={"auto": None, "on": True, "off": False}[args.letter_sum])
    W, parts, ms_per_step, value = run["W"], run["parts"], run["ms_per_step"], run["value"]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "reads/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f16", "fp8": "fp8e4m3"}[precision],
        "data": "synthetic",
        "config": {"workload": describe(w, precision, k, k_fetch, R, stride, radius, args.tokens),
                   "reads": R, "windows": W, "window_len": w.window_len,
                   "n_freq": tok.get("n_freq", w.n_freq), "tokens": args.tokens,
                   "stride": stride, "k": k, "k_fetch": k_fetch, "precision": precision,
                   "row_reals": run["row_reals"]},
        "window_scores_per_s": run["window_scores_per_s"],
        # the same step on an index built beforehand (reads -> product -> rescore)
        "reads_per_s_prebuilt_index": round(R / ((parts[1] + parts[2] + parts[3]) / 1e3), 1),
        "breakdown_ms": run["breakdown_ms"],
        "encoder_gbs": run["encoder_gbs"],
        "token_map_ms": None if token_map_ms is None else round(token_map_ms, 3),
        "accuracy": run["accuracy"],
        "roofline": run["roofline"],
    }
    low = [("headline", precision, value)]
    if (not args.no_fp8 and precision == "fp16" and not coarse and not wide
            and args.workload == "precision"):
        r8 = run_map(args, w, ref, reads, "fp8", k, k_fetch, stride, radius, tok,
                     max(1, args.steps), 1)
        out["fp8_path"] = {"value": round(r8["value"], 1), "unit": "reads/s",
                           "ms_per_step": round(r8["ms_per_step"], 3),
                           "breakdown_ms": r8["breakdown_ms"], "accuracy": r8["accuracy"],
                           "roofline": r8["roofline"], "row_reals": r8["row_reals"],
                           "note": "the same step with an FP8 e4m3 index and FP8 read heads "
                                   "(per-row FP32 scales), FP32 accumulation and FP32 rescore"}
        low.append(("fp8_path", "fp8", r8["value"]))
        if not args.no_fp8_letter_sum:
            r8s = run_map(args, w, ref, reads, "fp8", k, k_fetch, stride, radius, tok,
                          max(1, args.steps), 1, reduced=True)
            out["fp8_letter_sum_path"] = {
                "value": round(r8s["value"], 1), "unit": "reads/s",
                "ms_per_step": round(r8s["ms_per_step"], 3), "breakdown_ms": r8s["breakdown_ms"],
                "accuracy": r8s["accuracy"], "roofline": r8s["roofline"],
                "row_reals": r8s["row_reals"],
                "note": "the FP8 step with the index and read heads in the letter-sum form "
                        "(192 reals per row); not the library's FP8 default, since e4m3's "
                        "error per score grows by about sqrt(4/3) in it"}
            low.append(("fp8_letter_sum_path", "fp8", r8s["value"]))
    if (not args.no_threshold and args.workload == "precision" and not tok and not coarse):
        out["threshold_regime"] = threshold_leg(w, ref, reads, precision, args.threshold_err,
                                                floors=(0.0, args.threshold_floor))
    if not args.no_fp32 and precision != "fp32" and not coarse and not wide:
        fp = fp32_path(w, ref, reads, k, k_fetch, tok)
        fp["speedup_of_low_precision"] = {name: round(v / fp["value"], 2) for name, _, v in low}
        out["fp32_path"] = fp
        if not tok and not args.no_fp32_letter_sum:
            # the same algorithm in FP32: the letter-sum rows the FP16 headline uses
            fs = fp32_path(w, ref, reads, k, k_fetch, tok, reduced=True)
            fs["speedup_of_low_precision"] = {name: round(v / fs["value"], 2)
                                              for name, _, v in low}
            out["fp32_letter_sum_path"] = fs
    if not args.no_cpu_baseline:
        n_cpu = args.cpu_reads or {"scale": 1000}.get(w.name, 2000)
        out["cpu_baseline"] = cpu_baseline(w, ref, reads, W, n_cpu, args.cpu_windows,
                                           args.tokens)
    if (not args.no_batching and args.workload == "precision" and args.tokens is None
            and not coarse and args.reads is None):
        del reads
        b = bench_batching(args, fp32=not args.no_fp32, low=("fp16", "fp8"))
        out["batched_path"] = {key: b[key] for key in
                               ("value", "unit", "ms_per_step", "steps", "config",
                                "window_scores_per_s", "reads_per_s_prebuilt_index_eager",
                                "breakdown_ms_eager", "accuracy", "roofline", "fp8_path",
                                "fp8_letter_sum_path", "fp32_path") if key in b}
    print(json.dumps(out), flush=True)


def run_map(args, w, ref, reads, precision, k, k_fetch, stride, radius, tok, steps, warmup,
            reduced=None):
    """Build the index (reduced: the letter-sum form; None = the library's
    choice), then time `steps` whole steps (index build, read heads, product +
    top-k, FP32 rescore or refinement) with HIP events on torch's current
    stream; accuracy against the stored oracle lists.  The product's flops are
    those it executes: 4 per real of a row (K = 256, 192 in the letter-sum form,
    2,048 for 1,024-component tokens)."""
    import torch
    from paper_2603_22245_amd import mapper, _lib as L
    R = reads.n
    coarse = stride > w.stride
    wide = bool(tok) and 2 * tok["n_class"] * tok["n_freq"] != 256
    index = mapper.build_index(ref, window_len=w.window_len, stride=stride, precision=precision,
                               reanchor=w.reanchor, reduced=reduced, **tok)
    real_dim = index.real_dim
    flops_per_score = 4 * real_dim
    rb = mapper.upload_reads(index, reads.seq, reads.offsets)
    bufs = mapper.map_buffers(index, R, k, k_fetch)
    refine_ws = None
    if coarse:
        refine_ws = torch.empty(L.rm_refine_workspace_bytes(R, k_fetch, radius), dtype=torch.uint8,
                                device="cuda")
    torch.cuda.synchronize()
    W = index.n_windows
    log(f"index: W={W:,} precision={precision}; buffers ready")

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    ref_len = int(ref.shape[0])

    def step():
        ev[0].record()
        L.rm_encode_reference(index.ref, ref_len, index.params, index.buf, index.buf.numel())
        ev[1].record()
        mapper.encode_reads(index, rb)
        ev[2].record()
        mapper.score_topk(index, rb, bufs)
        ev[3].record()
        if coarse:
            mapper.refine(index, rb, bufs, radius, refine_ws)
        else:
            mapper.rescore(index, rb, bufs)
        ev[4].record()

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"{precision} warmup step {i + 1}/{warmup} done")
    parts = np.zeros(4)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(steps):
        step()
        torch.cuda.synchronize()
        parts += [ev[j].elapsed_time(ev[j + 1]) for j in range(4)]
        log(f"{precision} step {i + 1}/{steps}: "
            f"{sum(ev[j].elapsed_time(ev[j + 1]) for j in range(4)):.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / steps
    parts /= steps

    top_idx = bufs.top_idx.cpu().numpy()
    top_score = bufs.top_score.cpu().numpy()
    cand_idx = bufs.cand_idx.cpu().numpy()
    cand_score = bufs.cand_score.cpu().numpy()
    del index, rb, bufs, refine_ws
    torch.cuda.empty_cache()

    # ---- accuracy against the FP64 oracle
    # coarse candidates compared by their start (window id x stride)
    cand_start = np.where(cand_idx >= 0, cand_idx.astype(np.int64) * stride, -1)
    gold = None if not tok else f"{w.name}_{args.tokens}_top16_sample64.npz"
    acc = accuracy(w, reads, top_idx, top_score, cand_start, cand_score, k, R, gold, precision)

    # ---- dominant kernel: the scoring product (+ its small merge), HIP events
    score_s = parts[2] / 1e3
    achieved = R * W * flops_per_score / score_s / 1e12
    peak = PEAK_TFLOPS[precision]
    enc_bytes = W * (real_dim * {"fp32": 4, "fp16": 2, "fp8": 1}[precision] + 8) + ref_len
    traffic = None
    if R == w.n_reads and not coarse and (not tok or wide):
        traffic = measured_traffic(w.name, precision, args.tokens,
                                   None if args.tokens else real_dim)
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel": ("score_wide_kernel (+merge_wide_kernel)" if wide
                           else "score_topk_kernel (+merge_kernel)"),
                "algorithmic": f"{flops_per_score} flops per (read, window) score x {R} x {W}"}
    return {"W": W, "parts": parts, "ms_per_step": ms_per_step, "value": R / (ms_per_step / 1e3),
            "row_reals": real_dim,
            "window_scores_per_s": float(f"{R * W / score_s:.4g}"),
            "breakdown_ms": {"encode_reference": round(parts[0], 3),
                             "encode_reads": round(parts[1], 3),
                             "score_topk": round(parts[2], 3),
                             ("refine" if coarse else "rescore"): round(parts[3], 3)},
            "encoder_gbs": round(enc_bytes / (parts[0] / 1e3) / 1e9, 1),
            "accuracy": acc, "roofline": roofline}


def _batched_pass(ref, reads, k, k_fetch, precision, steps, warmup, reduced=None):
    """Bucket indexes, the autotuned grouped persistent scoring launch, and the
    whole step (index builds, read heads, product + top-k, FP32 rescore)
    captured in a HIP graph and replayed `steps` times; returns the mapper (to
    read results from) and the timings."""
    import torch
    from paper_2603_22245_amd import mapper
    bm = mapper.BatchMapper(ref, reads.seq, reads.offsets, k=k, k_fetch=k_fetch,
                            precision=precision, reduced=reduced)
    stream = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    with torch.cuda.stream(stream):
        bm.encode(stream)
        torch.cuda.synchronize()
        best, tuned_ms = bm.autotune(os.environ.get("RM_AUTOTUNE_CACHE"), stream)
        log(f"{precision} autotune: read_tile={best.read_tile} chunk_tiles={best.chunk_tiles} "
            f"({tuned_ms:.2f} ms)")
        # one eager pass with events for the breakdown
        ev[0].record(stream)
        bm.rebuild_indexes(stream)
        ev[1].record(stream)
        bm.encode(stream)
        ev[2].record(stream)
        bm.score(stream)
        ev[3].record(stream)
        bm.rescore(stream)
        ev[4].record(stream)
        stream.synchronize()
        parts = [ev[j].elapsed_time(ev[j + 1]) for j in range(4)]
        bm.capture(stream, with_index=True)
        for i in range(warmup):
            bm.replay(stream)
            stream.synchronize()
            log(f"{precision} warmup replay {i + 1}/{warmup} done")
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for i in range(steps):
            bm.replay(stream)
            stream.synchronize()
            log(f"{precision} replay {i + 1}/{steps} done")
        wall = time.perf_counter() - t_start
    return bm, wall * 1e3 / steps, parts, best


def bench_batching(args, fp32: bool = None, low=None):
    """Reads of uneven length: bucket indexes, one grouped persistent scoring launch,
    the whole step replayed from a HIP graph; then the same step with FP32
    indexes and the FP32 product (the plain FP32 path) for comparison.  `low`:
    (headline precision, another low precision run as a second leg)."""
    import torch
    import synth
    w = synth.WORKLOADS["batching"]
    precision = args.precision or w.precision
    if low is not None:
        precision = low[0]
    k, k_fetch = w.k, max(w.k, args.k_fetch)
    fp32 = (not args.no_fp32) if fp32 is None else fp32
    t0 = time.time()
    ref = w.reference()
    reads = w.reads(ref)
    if args.workload == "batching" and args.reads is not None and args.reads < reads.n:
        n = args.reads
        reads = synth.Reads(reads.seq[:reads.offsets[n]], reads.offsets[:n + 1], reads.truth[:n])
    R = reads.n
    log(f"workload batching: G={ref.shape[0]:,} R={R:,} generated in {time.time() - t0:.1f}s")
    bm, ms_per_step, parts, best = _batched_pass(ref, reads, k, k_fetch, precision, args.steps,
                                                 args.warmup)
    value = R / (ms_per_step / 1e3)
    scores = sum(b.reads.n * b.index.n_windows for b in bm.buckets)
    # flops the product executes: 4 per real of the buckets' rows
    flops = sum(b.reads.n * b.index.n_windows * 4 * b.index.real_dim for b in bm.buckets)
    row_reals = sorted({b.index.real_dim for b in bm.buckets})
    peak = PEAK_TFLOPS[precision]
    achieved = flops / (parts[2] / 1e3) / 1e12
    ids, sc = bm.results()
    acc = batching_accuracy(ref, reads, bm, ids, sc, k)
    buckets = [{"N": b.length, "stride": b.stride, "reads": int(b.reads.n),
                "windows": int(b.index.n_windows)} for b in bm.buckets]
    bm.close()
    del bm
    torch.cuda.empty_cache()
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "reads/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f16", "fp8": "fp8e4m3"}[precision], "data": "synthetic",
        "config": {"workload": (f"batching: 64 Mbp synthetic reference (45% GC, 8% repeats), "
                                f"{R:,} reads of lognormal length (median 2 kbp, 100 bp-10 kbp), "
                                f"5-10% indel-heavy error; buckets N_b = 100..6400 bp at stride "
                                f"N_b/100; one persistent {precision} scoring launch; the step "
                                f"(index builds, encode, score, rescore) replayed from a HIP graph"),
                   "reads": R, "buckets": buckets, "k": k, "k_fetch": k_fetch,
                   "precision": precision,
                   "tuning": {"read_tile": best.read_tile, "chunk_tiles": best.chunk_tiles}},
        "window_scores_per_s": float(f"{scores / (parts[2] / 1e3):.4g}"),
        "reads_per_s_prebuilt_index_eager": round(R / ((parts[1] + parts[2] + parts[3]) / 1e3), 1),
        "breakdown_ms_eager": {"encode_references": round(parts[0], 3),
                               "encode_reads": round(parts[1], 3),
                               "score_topk_grouped": round(parts[2], 3),
                               "rescore": round(parts[3], 3)},
        "accuracy": acc,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                     "kernel": "score_topk_kernel (grouped, persistent) + merges",
                     "algorithmic": f"4 flops per real of rows of {row_reals} reals x {scores} "
                                    f"(read, window) scores"},
    }
    prebuilt = {precision: parts[1] + parts[2] + parts[3]}
    step_ms = {precision: ms_per_step}
    # further low-precision legs: (precision, row form, output key)
    legs = []
    if low is not None and len(low) > 1:
        legs.append((low[1], None, f"{low[1]}_path"))
        if low[1] == "fp8" and not getattr(args, "no_fp8_letter_sum", False):
            legs.append(("fp8", True, "fp8_letter_sum_path"))
    for p2, red2, key2 in legs:
        bm2, ms2, parts2, best2 = _batched_pass(ref, reads, k, k_fetch, p2, args.steps, 1,
                                                reduced=red2)
        flops2 = sum(b.reads.n * b.index.n_windows * 4 * b.index.real_dim for b in bm2.buckets)
        rr2 = sorted({b.index.real_dim for b in bm2.buckets})
        ids2, sc2 = bm2.results()
        acc2 = batching_accuracy(ref, reads, bm2, ids2, sc2, k)
        bm2.close()
        del bm2
        torch.cuda.empty_cache()
        name2 = key2[:-len("_path")]
        prebuilt[name2] = parts2[1] + parts2[2] + parts2[3]
        step_ms[name2] = ms2
        out[key2] = {
            "value": round(R / (ms2 / 1e3), 1), "unit": "reads/s", "ms_per_step": round(ms2, 3),
            "reads_per_s_prebuilt_index_eager": round(R / (prebuilt[name2] / 1e3), 1),
            "breakdown_ms_eager": {"encode_references": round(parts2[0], 3),
                                   "encode_reads": round(parts2[1], 3),
                                   "score_topk_grouped": round(parts2[2], 3),
                                   "rescore": round(parts2[3], 3)},
            "accuracy": acc2,
            "roofline": {"bound": "mfma",
                         "achieved": round(flops2 / (parts2[2] / 1e3) / 1e12, 2),
                         "peak": PEAK_TFLOPS[p2], "unit": "TFLOP/s",
                         "frac": round(flops2 / (parts2[2] / 1e3) / 1e12 / PEAK_TFLOPS[p2], 4),
                         "traffic": None},
            "row_reals": rr2,
            "note": f"the same graph-replayed step with {p2} indexes and read heads"
                    f"{' in the letter-sum form' if red2 else ''} "
                    f"(tuning read_tile={best2.read_tile}, chunk_tiles={best2.chunk_tiles})"}
    if fp32 and precision != "fp32":
        bm32, ms32, parts32, best32 = _batched_pass(ref, reads, k, k_fetch, "fp32", 1, 1)
        ids32, sc32 = bm32.results()
        acc32 = batching_accuracy(ref, reads, bm32, ids32, sc32, k)
        bm32.close()
        del bm32
        torch.cuda.empty_cache()
        v32 = R / (ms32 / 1e3)
        out["fp32_path"] = {
            "value": round(v32, 1), "unit": "reads/s", "ms_per_step": round(ms32, 3),
            "tflops": round(scores * FLOPS_PER_SCORE / (parts32[2] / 1e3) / 1e12, 2),
            "breakdown_ms_eager": {"encode_references": round(parts32[0], 3),
                                   "encode_reads": round(parts32[1], 3),
                                   "score_topk_grouped": round(parts32[2], 3),
                                   "rescore": round(parts32[3], 3)},
            "accuracy": acc32,
            "speedup_of_low_precision": {p: round(ms32 / t, 2) for p, t in step_ms.items()},
            "speedup_of_low_precision_prebuilt_index": {
                p: round((parts32[1] + parts32[2] + parts32[3]) / t, 2)
                for p, t in prebuilt.items()},
            "note": "the same graph-replayed step with FP32 indexes and the FP32 MFMA product "
                    f"(tuning read_tile={best32.read_tile}, chunk_tiles={best32.chunk_tiles})"}
    return out


def _spearman(x, y) -> float:
    from scipy.stats import spearmanr
    return float(spearmanr(x, y).correlation)


def bench_correlation(args):
    """The correlation protocol of §2.4 on the GPU: random 150 bp strings and
    companions mutated at rates err evenly spread over (0, 0.5) (edits split
    evenly between substitutions, insertions and deletions), their fidelities
    under the plain and the learned encoding, the fitting curve and the RMSE of
    predicting err from the fidelity."""
    import torch
    import synth
    from paper_2603_22245_amd import correlation as CR, learned as LM
    N, levels = 150, 25
    per = max(1, args.corr_pairs // levels)
    err_levels = (np.arange(levels) + 0.5) * 0.5 / levels
    edits = np.repeat(np.rint(err_levels * N).astype(np.int64), per)
    t0 = time.time()
    pairs = synth.mutate_pairs(edits.size, N, int(edits.max()), seed=403, edits=edits)
    log(f"correlation: {pairs.n:,} pairs at {levels} mutation rates generated in "
        f"{time.time() - t0:.1f}s")
    ps = LM.upload_pairs(pairs.a, pairs.a_off, pairs.b, pairs.b_off)
    weights = np.load(os.path.join(ROOT, "tests", "golden", "learned_weights.npy"))
    params = torch.from_numpy(weights.astype(np.float32)).cuda()
    out_F = {}
    ms = {}
    for name, prm in (("plain", None), ("learned", params)):
        CR.run(ps, err_levels, N, prm)          # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        F, E, rmse = CR.run(ps, err_levels, N, prm)
        e1.record()
        torch.cuda.synchronize()
        ms[name] = e0.elapsed_time(e1)
        out_F[name] = (E.cpu().numpy().astype(np.float64), rmse.cpu().numpy().astype(np.float64))
    res = {}
    for name, (E, rmse) in out_F.items():
        low = err_levels < 0.25
        res[name] = {"E_fid": [round(float(v), 5) for v in E],
                     "rmse": [round(float(r), 5) for r in rmse],
                     "max_rmse_below_25pct": round(float(np.max(rmse[low])), 5),
                     "mean_rmse": round(float(np.mean(rmse)), 5)}
    value = pairs.n / (ms["plain"] / 1e3)
    return {
        "metric": "pair fidelities/s (plain encoding); RMSE of predicting the mutation rate "
                  "from fidelity (§2.4 protocol)",
        "value": round(value, 1), "unit": "pairs/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(ms["plain"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"correlation: {pairs.n:,} pairs of a uniform {N} bp string and "
                               f"its companion after round(err N) edits (substitution, insertion, "
                               f"deletion uniform), err at {levels} rates evenly over (0, 0.5), "
                               f"{per} pairs per rate; plain and learned (stored weights) "
                               f"encodings, m=32",
                   "pairs": pairs.n, "window_len": N, "levels": levels},
        "err_levels": [round(float(e), 4) for e in err_levels],
        "plain": res["plain"], "learned": res["learned"],
        "learned_ms": round(ms["learned"], 3),
    }


def bench_learned(args):
    """The learned offsets: edit-distance labels, GPU training (time per epoch),
    held-out Spearman correlation with edit distance (learned vs plain), then
    the precision workload mapped with the learned encoding."""
    import torch
    import synth
    from paper_2603_22245_amd import learned as LM
    n_pairs = args.pairs
    n_train = int(round(0.9 * n_pairs))
    t0 = time.time()
    P = synth.mutate_pairs(n_pairs, 150, 30, seed=synth.PAIRS_SEED)
    log(f"learned: {n_pairs:,} pairs generated in {time.time() - t0:.1f}s")
    full = LM.upload_pairs(P.a, P.a_off, P.b, P.b_off)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    LM.levenshtein(full)  # warm-up
    ev[0].record()
    ld = LM.levenshtein(full)
    ev[1].record()
    torch.cuda.synchronize()
    lev_ms = ev[0].elapsed_time(ev[1])
    full.ld = ld

    def part(i0, i1):
        return LM.PairSet(full.a, full.a_off[i0:i1 + 1], full.b, full.b_off[i0:i1 + 1], i1 - i0,
                          full.ld[i0:i1])

    train, held = part(0, n_train), part(n_train, n_pairs)
    ld_held = held.ld.cpu().numpy()
    N = 150
    rho = {"plain_whole_string": _spearman(LM.pair_fidelity(None, held, N).cpu().numpy(), -ld_held),
           "plain_token_middles": _spearman(
               LM.pair_fidelity(torch.from_numpy(LM.init_params(0)).cuda(), held,
                                N).cpu().numpy(), -ld_held)}
    t = LM.Trainer(seed=0, batch=1024, lr=3e-3)
    epochs = []
    for ep in range(args.epochs):
        torch.cuda.synchronize()
        a = time.perf_counter()
        losses = t.epoch(train, graph=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - a
        lo = losses.cpu().numpy()
        r = _spearman(LM.pair_fidelity(t.params, held, N).cpu().numpy(), -ld_held)
        epochs.append({"seconds": round(dt, 3), "first_loss": round(float(lo[:16].mean()), 4),
                       "last_loss": round(float(lo[-16:].mean()), 4),
                       "heldout_spearman": round(r, 4),
                       "note": "includes graph capture" if ep == 0 else "graph replay"})
        log(f"epoch {ep}: {dt:.3f}s loss {lo[:16].mean():.4f} -> {lo[-16:].mean():.4f}, "
            f"held-out Spearman {r:.4f}")
    steps = n_train // 1024
    rep = [e["seconds"] for e in epochs[1:]] or [epochs[0]["seconds"]]
    epoch_s = float(np.median(rep))
    rho["learned_gpu_trained"] = epochs[-1]["heldout_spearman"]
    wpath = os.path.join(ROOT, "tests", "golden", "learned_weights.npy")
    stored = np.load(wpath) if os.path.exists(wpath) else None
    if stored is not None:
        rho["learned_cpu_oracle_trained"] = round(_spearman(
            LM.pair_fidelity(torch.from_numpy(stored).cuda(), held, N).cpu().numpy(), -ld_held), 4)
    out = {
        "metric": "training pairs/s (FP32, one GPU); held-out Spearman vs edit distance",
        "value": round(steps * 1024 / epoch_s, 1), "unit": "pairs/s", "n_gpus": 1,
        "steps": steps * len(epochs), "warmup": 0, "ms_per_step": round(epoch_s * 1e3 / steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"learned: {n_pairs:,} pairs (a uniform 150 bp, b = a after "
                                f"0-30 random edits), exact edit-distance labels; MLP 32-64-128 "
                                f"(10,432 parameters), FP32 training, batches of 1024, Adam "
                                f"lr 3e-3; {n_train:,} train / {n_pairs - n_train:,} held out"),
                   "pairs": n_pairs, "epochs": len(epochs)},
        "epoch_seconds": epoch_s, "epochs": epochs,
        "levenshtein": {"ms": round(lev_ms, 3), "pairs_per_s": float(f"{n_pairs / lev_ms * 1e3:.4g}")},
        "spearman_vs_minus_ld": {k: round(v, 4) for k, v in rho.items()},
    }
    t.close()
    del t, full, train, held
    torch.cuda.empty_cache()
    if not args.no_map_rerun:
        weights = stored if stored is not None else None
        out["precision_rerun_learned"] = learned_map_rerun(args, weights)
    return out


def learned_map_rerun(args, weights):
    """The precision workload mapped with the learned encoding (BF16 offsets):
    offsets of the reference + rolling index, offsets of the reads + read heads,
    the unchanged scoring launch, FP32 rescore with offsets."""
    import torch
    import synth
    from paper_2603_22245_amd import mapper, learned as LM
    w = synth.WORKLOADS["precision"]
    precision = args.precision or w.precision
    k, k_fetch = w.k, max(w.k, args.k_fetch)
    src = "weights trained by the CPU oracle (tests/golden/learned_weights.npy)"
    if weights is None:
        weights, src = LM.init_params(0), "untrained network (stored weights missing)"
    ref = w.reference()
    reads = w.reads(ref)
    if args.reads is not None and args.reads < reads.n:
        n = args.reads
        reads = synth.Reads(reads.seq[:reads.offsets[n]], reads.offsets[:n + 1], reads.truth[:n])
    R = reads.n
    index = mapper.build_index(ref, window_len=w.window_len, stride=w.stride, precision=precision,
                               reanchor=w.reanchor, learned=weights)
    rb = mapper.upload_reads(index, reads.seq, reads.offsets)
    bufs = mapper.map_buffers(index, R, k, k_fetch)
    torch.cuda.synchronize()
    from paper_2603_22245_amd import _lib as L
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    G = int(ref.shape[0])

    def step():
        ev[0].record()
        L.rm_mlp_infer(index.learned, index.ref, G, index.delta)
        ev[1].record()
        L.rm_encode_reference_learned(index.ref, G, index.params, index.delta, index.buf,
                                      index.buf.numel())
        ev[2].record()
        mapper.encode_reads(index, rb)
        ev[3].record()
        mapper.score_topk(index, rb, bufs)
        ev[4].record()
        mapper.rescore(index, rb, bufs)
        ev[5].record()

    step()
    torch.cuda.synchronize()
    parts = np.zeros(5)
    a = time.perf_counter()
    for i in range(args.steps):
        step()
        torch.cuda.synchronize()
        parts += [ev[j].elapsed_time(ev[j + 1]) for j in range(5)]
        log(f"learned rerun step {i + 1}/{args.steps}")
    dt = (time.perf_counter() - a) / args.steps
    parts /= args.steps
    acc = accuracy(w, reads, bufs.top_idx.cpu().numpy(), bufs.top_score.cpu().numpy(),
                   bufs.cand_idx.cpu().numpy(), bufs.cand_score.cpu().numpy(), k, R,
                   gold_name="precision_learned_top16_sample64.npz")
    W = index.n_windows
    infer_bytes = (G - 8) * 128 + G
    res = {"value": round(R / dt, 1), "unit": "reads/s", "ms_per_step": round(dt * 1e3, 3),
           "precision": precision, "weights": src, "reads": R, "windows": W,
           "breakdown_ms": {"mlp_infer_reference": round(parts[0], 3),
                            "encode_reference_learned": round(parts[1], 3),
                            "encode_reads_learned (incl. their offsets)": round(parts[2], 3),
                            "score_topk": round(parts[3], 3), "rescore_learned": round(parts[4], 3)},
           "mlp_infer_gbs": round(infer_bytes / (parts[0] / 1e3) / 1e9, 1),
           "score_tflops": round(R * W * FLOPS_PER_SCORE / (parts[3] / 1e3) / 1e12, 1),
           "accuracy": acc}
    del index, rb, bufs
    torch.cuda.empty_cache()
    return res


TIE_TAU = 1e-5   # oracle fidelities closer than this count as tied


def score_vs_stored(got_idx, got_F, gold_idx, gold_F, k, tau=TIE_TAU):
    """Recall@k and exact-list agreement of one read's list against the oracle's
    stored ranked list (longer than k).  A window outside the stored list has a
    true fidelity at most the stored list's last one and is counted as a miss
    (conservative); for windows in it the stored fidelity is the true one.
    Returns (recall, exact, max |score - stored F| over windows in the list)."""
    pos = {int(j): i for i, j in enumerate(gold_idx)}
    Fk = gold_F[k - 1]
    top = set(int(j) for j in gold_idx[:k])
    hits, ranks_ok, err = 0, True, 0.0
    seen = set()
    for r, j in enumerate(got_idx[:k]):
        j = int(j)
        if j in seen or j not in pos:
            ranks_ok = False
            continue
        seen.add(j)
        Fj = gold_F[pos[j]]
        err = max(err, abs(float(got_F[r]) - Fj))
        if j in top or Fj >= Fk - tau:
            hits += 1
        if abs(Fj - gold_F[r]) > tau:
            ranks_ok = False
    return hits / k, ranks_ok, err


def batching_accuracy(ref, reads, bm, ids, sc, k):
    res = {"unmapped_reads": int(np.sum(bm.bucket_of < 0))}
    gold = os.path.join(ROOT, "tests", "golden", "batching_top16_per_bucket4.npz")
    if not os.path.exists(gold):
        res["recall_at_k"] = None
        return res
    g = np.load(gold)
    recs, exact, errs = [], [], []
    for r, oi, of in zip(g["reads"], g["idx"], g["F"]):
        if r >= reads.n:
            continue
        rec, ex, e = score_vs_stored(ids[r], sc[r], oi, of, k)
        recs.append(rec)
        exact.append(ex)
        errs.append(e)
    res["recall_at_k"] = round(float(np.mean(recs)), 5) if recs else None
    res["exact_lists_up_to_ties"] = round(float(np.mean(exact)), 5) if exact else None
    res["rescore_max_abs_err"] = float(f"{max(errs):.3g}") if errs else None
    res["sample_reads"] = len(recs)
    res["reference"] = "oracle top-16 lists stored in tests/golden"
    return res


def describe(w, precision, k, k_fetch, R, stride=None, radius=0, tokens=None):
    stride = w.stride if stride is None else stride
    enc = f"m={w.n_freq}"
    if tokens is not None:
        import synth
        s, m, C, tm, sched = synth.token_encoding(tokens)
        kept = (f", the {C} most frequent kept" if synth.token_map_is_frequent(tokens) else
                f" mapped to {C} classes" if tm is not None else "")
        enc = f"{s}-mer tokens{kept}, m={m}, {sched} factors"
    head = (f"{w.name}: {w.G / 1e6:g} Mbp synthetic reference ({int(w.gc * 100)}% GC, "
            f"{int(w.repeat_frac * 100)}% repeats), {R:,} reads of {w.read_len} bp, N={w.window_len}, "
            f"{enc}, stride {stride}, {precision} index, ")
    if stride > w.stride:
        return head + (f"top-{k_fetch} coarse windows refined in FP32 over the step-1 windows "
                       f"within {radius} letters, top-{k} kept")
    return head + f"top-{k} of {k_fetch} rescored in FP32"


PRODUCT_TOL = {"fp32": 1e-5, "fp16": 1e-3, "fp8": 1e-2}   # relative bounds on the product's F


def _gold_file(w, gold_name=None):
    """The stored oracle sample of a workload: the named file, else the
    largest stored sample (top-32 of 2,000 precision reads or 1,000 scale
    reads), else the 64-read top-16 one."""
    base = os.path.join(ROOT, "tests", "golden")
    names = [gold_name] if gold_name else [f"{w.name}_top32_sample2000.npz",
                                           f"{w.name}_top32_sample1000.npz",
                                           f"{w.name}_top16_sample64.npz"]
    for n in names:
        if os.path.exists(os.path.join(base, n)):
            return os.path.join(base, n)
    return None


def accuracy(w, reads, top_idx, top_score, cand_idx, cand_score, k, R, gold_name=None,
             precision=None):
    """Recall@k and score errors against the oracle's stored sample; true-location rate.
    The product's scores of candidates found in the stored lists are checked
    against |dF| <= tol max(F, F_best) (tol 1e-3 FP16, 1e-2 FP8; F_best the
    read's best oracle score) and the fraction inside is reported."""
    res = {}
    # true location: the read's sampled start within a few windows of the top-1
    truth_win = reads.truth // w.stride
    res["top1_within_8_of_truth"] = round(float(np.mean(np.abs(top_idx[:, 0] - truth_win) <= 8)), 5)
    gold = _gold_file(w, gold_name)
    if gold is None:
        res["recall_at_k"] = None
        return res
    g = np.load(gold)
    pick = g["reads"]
    if pick.max() >= R:
        res["recall_at_k"] = None
        res["note"] = f"the stored sample's reads lie beyond the first {R:,} reads"
        return res
    recs, exact, errs, perr, prel, inside = [], [], [], [], [], []
    tol = PRODUCT_TOL.get(precision)
    for r, oi, of in zip(pick, g["idx"], g["F"]):
        rec, ex, e = score_vs_stored(top_idx[r], top_score[r], oi, of, k)
        recs.append(rec)
        exact.append(ex)
        errs.append(e)
        # low-precision product scores of candidates found in the stored list
        pos = {int(j): i for i, j in enumerate(oi)}
        for j, sc in zip(cand_idx[r], cand_score[r]):
            if int(j) in pos:
                Fj = of[pos[int(j)]]
                perr.append(abs(float(sc) - Fj))
                prel.append(abs(float(sc) - Fj) / max(Fj, of[0]))
                if tol is not None:
                    inside.append(abs(float(sc) - Fj) <= tol * max(Fj, of[0]))
    res["recall_at_k"] = round(float(np.mean(recs)), 5)
    res["exact_lists_up_to_ties"] = round(float(np.mean(exact)), 5)
    res["rescore_max_abs_err"] = float(f"{max(errs):.3g}")
    res["product_max_abs_err"] = float(f"{max(perr):.3g}") if perr else None
    res["product_max_rel_err_vs_best"] = float(f"{max(prel):.3g}") if prel else None
    if inside:
        res["product_scores_checked"] = len(inside)
        res["product_frac_within_rel_bound"] = round(float(np.mean(inside)), 6)
        res["product_rel_bound"] = tol
    res["sample_reads"] = int(pick.shape[0])
    res["reference"] = f"oracle top-{g['idx'].shape[1]} lists stored in tests/golden/" \
                       f"{os.path.basename(gold)}"
    return res


def location_clusters(ids, span):
    """Distinct locations among a read's window ids: windows whose ids differ
    by at most `span` (windows that overlap the same stretch of reference)
    form one location.  Returns the number of such clusters."""
    ids = np.sort(np.asarray(ids, dtype=np.int64))
    if ids.size == 0:
        return 0
    return int(1 + np.count_nonzero(np.diff(ids) > span))


def threshold_leg(w, ref, reads, precision, err, copies=16, rank=1, seed=1, floors=(0.0,)):
    """§3.3 / §3.5: per-window thresholds at a target mutation rate (the
    rank-th smallest fidelity of `copies` mutated copies of each window), then
    every location whose FP32 fidelity passes max(its window's threshold,
    floor), for every read, once per floor.  Reports, per floor, windows and
    distinct places per read, the share of reads with exactly one place, and the
    share whose windows miss the read's true window (within 8 windows); and the
    thresholds' low percentiles (a window whose mutated copies can lose their
    alignment to net indels gets a threshold near 0, and every read passes it)."""
    import torch
    from paper_2603_22245_amd import mapper
    index = mapper.build_index(ref, window_len=w.window_len, stride=w.stride, precision=precision,
                               reanchor=w.reanchor)
    rb = mapper.upload_reads(index, reads.seq, reads.offsets)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    mapper.window_thresholds(index, err, copies, rank, seed)            # warm-up
    torch.cuda.synchronize()
    ev[0].record()
    thr = mapper.window_thresholds(index, err, copies, rank, seed)
    ev[1].record()
    mapper.encode_reads(index, rb)
    torch.cuda.synchronize()
    thr_ms = ev[0].elapsed_time(ev[1])
    thr_h = thr.cpu().numpy()
    truth = reads.truth // w.stride
    # at stride 1 a read passes the thresholds of many overlapping windows
    # around one place; count places: windows overlapping one another (ids
    # within a window length) are one location
    span = max(1, w.window_len // w.stride)
    runs = []
    for floor in floors:
        h = mapper.score_threshold(index, rb, thr, floor)                # sizes the capacity
        torch.cuda.synchronize()
        ev[2].record()
        h = mapper.score_threshold(index, rb, thr, floor, capacity=h.capacity)
        ev[3].record()
        torch.cuda.synchronize()
        regime_ms = ev[2].elapsed_time(ev[3])
        n = h.n_found.cpu().numpy()
        lists = h.lists()
        hit = np.array([np.any(np.abs(ids.astype(np.int64) - t) <= 8) for (ids, _), t in
                        zip(lists, truth)])
        loc = np.array([location_clusters(ids, span) for ids, _ in lists])
        del h
        log(f"threshold regime, floor {floor}: {regime_ms:.1f} ms")
        runs.append({"floor": floor, "regime_ms": round(regime_ms, 3),
                     "reads_per_s": round(reads.n / (regime_ms / 1e3), 1),
                     "windows_per_read": round(float(n.mean()), 3),
                     "max_windows": int(n.max()),
                     "locations_per_read": round(float(loc.mean()), 3),
                     "max_locations": int(loc.max()),
                     "mapped_to_one_location": round(float(np.mean(loc == 1)), 4),
                     "unmapped": round(float(np.mean(n == 0)), 4),
                     "missed_true_location": round(float(np.mean(~hit)), 4)})
    del index, rb, thr
    torch.cuda.empty_cache()
    log(f"threshold regime: {thr_ms:.1f} ms thresholds")
    return {"target_err": err, "copies": copies, "rank": rank, "precision": precision,
            "thresholds_ms": round(thr_ms, 3),
            "threshold_percentiles": {str(q): round(float(np.percentile(thr_h, q)), 4)
                                      for q in (0.1, 1, 5, 50)},
            "runs": runs,
            "note": "regime: read heads encoded beforehand; MFMA proposal pass + grouping + "
                    "FP32 recompute of the proposals; thresholds timed separately"}


def fp32_path(w, ref, reads, k, k_fetch, tok=None, reduced=False):
    """Timed whole steps of the plain FP32 path: the same step (index build,
    read heads, product + top-k, FP32 rescore) with an FP32 index and the FP32
    MFMA product; full rows, or with reduced=True the letter-sum form."""
    import torch
    from paper_2603_22245_amd import mapper, _lib as L
    index = mapper.build_index(ref, window_len=w.window_len, stride=w.stride, precision="fp32",
                               reanchor=w.reanchor, reduced=reduced, **(tok or {}))
    row_reals = index.real_dim
    rb = mapper.upload_reads(index, reads.seq, reads.offsets)
    bufs = mapper.map_buffers(index, reads.n, k, k_fetch)
    ref_len = int(ref.shape[0])

    def step():
        L.rm_encode_reference(index.ref, ref_len, index.params, index.buf, index.buf.numel())
        mapper.map_reads(index, rb, bufs)

    step()  # warm-up / first launch
    torch.cuda.synchronize()
    t = time.perf_counter()
    step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    v = reads.n / dt
    log(f"fp32 path: {dt * 1e3:.1f} ms per step")
    W = index.n_windows
    top_idx = bufs.top_idx.cpu().numpy()
    top_score = bufs.top_score.cpu().numpy()
    cand_idx = bufs.cand_idx.cpu().numpy()
    cand_score = bufs.cand_score.cpu().numpy()
    del index, rb, bufs
    torch.cuda.empty_cache()
    acc = accuracy(w, reads, top_idx, top_score, cand_idx, cand_score, k, reads.n,
                   precision="fp32")
    return {"value": round(v, 1), "unit": "reads/s", "ms_per_step": round(dt * 1e3, 2),
            "row_reals": row_reals,
            "tflops": round(reads.n * W * 4 * row_reals / dt / 1e12, 2),
            "accuracy": {key: acc.get(key) for key in ("recall_at_k", "exact_lists_up_to_ties",
                                                       "sample_reads")},
            "note": f"index build + read encoding + FP32 MFMA product over rows of "
                    f"{row_reals} reals + top-k + FP32 rescore (tflops over the whole step)"}


def cpu_baseline(w, ref, reads, W, n_reads, n_windows, tokens_name=None):
    """The FP64 oracle mapping a bounded sample: n_reads read heads (those of the
    stored oracle sample when there is one) against the first n_windows windows
    (direct encoding + brute-force scan), scaled to all windows."""
    from oracle import mapping, tokens
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count()
    nw = min(n_windows, W)
    # the stored oracle sample's reads (recall is reported on them), else the first reads
    gold = _gold_file(w) if tokens_name is None else None
    pick = np.arange(min(n_reads, reads.n))
    if gold is not None:
        g = np.load(gold)["reads"]
        if g.max() < reads.n:
            pick = g[:n_reads]
    n_reads = int(pick.size)
    heads = mapping.read_heads(reads.seq, reads.offsets, w.window_len)[pick]
    t = time.perf_counter()
    if tokens_name is None:
        mapping.map_reads(ref, heads, w.window_len, w.n_freq, w.k, w.stride, window_range=(0, nw))
    else:
        import synth
        s, m, C, tm, sched = synth.token_encoding(tokens_name)
        if synth.token_map_is_frequent(tokens_name):
            tm = tokens.frequent_map(ref, s, C)
        tokens.map_reads(ref, heads, w.window_len, s, m, C, tm, w.k, w.stride, sched,
                         window_range=(0, nw))
    dt = time.perf_counter() - t
    v = n_reads / dt * (nw / W)
    log(f"cpu baseline: {n_reads} reads x {nw:,} windows in {dt:.1f}s")
    # the same oracle on one thread, over a quarter of the windows
    nw1 = max(1, nw // 4)
    v1 = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t = time.perf_counter()
            if tokens_name is None:
                mapping.map_reads(ref, heads, w.window_len, w.n_freq, w.k, w.stride,
                                  window_range=(0, nw1))
            else:
                tokens.map_reads(ref, heads, w.window_len, s, m, C, tm, w.k, w.stride, sched,
                                 window_range=(0, nw1))
            v1 = n_reads / (time.perf_counter() - t) * (nw1 / W)
    except ImportError:
        pass
    out = {"value": float(f"{v:.4g}"), "unit": "reads/s", "cores": cores, "kind": "oracle",
           "sample": f"{n_reads} read heads x first {nw:,} of {W:,} windows (FP64 encoding + "
                     f"brute-force scan, {dt:.1f} s), scaled by {nw:,}/{W:,}",
           "host_cpus": os.cpu_count(), "cpu_model": _cpu_model(), "ram_gib": _ram_gib()}
    if v1 is not None:
        out["single_thread_value"] = float(f"{v1:.4g}")
        out["single_thread_sample"] = f"the same reads x first {nw1:,} windows on one thread"
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _ram_gib():
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    return round(int(line.split()[1]) / 2**20, 1)
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
