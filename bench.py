#!/usr/bin/env python3
"""Benchmark of the PixelBox hot path on one MI355X.

Workload (default): the heavy-tailed mix -- 2,000,000 polygon pairs whose MBR
side is lognormal (median 24 px, clipped to 8-400 px), 1% of them merged
blobs of 10-40 ellipses -- synthetic and seeded, resident in HBM before the
timed region.  One step = one sccg_area_pairs call in BATCHED mode over all
pairs (per-pair MBRs and areas, pair boxes, sampling-box splits, leaf
crossing tests, int64 intersection and union counts), launched as one
captured HIP graph around one persistent kernel.

Printed: one JSON line with pairs/s (the value), pixel-tests/s, the plain
one-pair-per-workgroup kernel's pairs/s on the same pairs, the roofline of
the persistent kernel, and the CPU oracle's rate on a bounded sample.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "polygon pairs/sec and pixel-tests/sec, bit-exact; batched vs plain kernel"

WORKLOADS = {
    6: "Figure 8 stand-in: 15,724 uniform-mix pairs with coordinates scaled by k = 1..5; PixelOnly, "
       "PixelBox-NoSep and PixelBox (batched) and the plain Algorithm 1 kernel, each autotuned",
    5: "serving: Poisson job arrivals at 5, 20 and 80 jobs/s, 600 jobs per rate (first 20 not measured), "
       "each job a window of 1e3-5e5 pairs (log-uniform) of a pinned 500,000-pair uniform-mix corpus",
    4: "set-level: 64 tiles of 8192^2 px, per tile set A of 10-60 px shapes packed pixel-disjoint (skyline "
       "drop, 37.7k per tile) and set B = 85% shifted "
       "and dilated/eroded copies + 15% fresh shapes, candidate pairs from a 64-px grid MBR join; "
       "step = pair counts + per-tile Jaccard",
    3: "heavy-tailed mix: 2,000,000 pairs, MBR side lognormal (median 24 px, clipped 8-400 px), "
       "1% merged blobs of 10-40 ellipses, one persistent launch",
    2: "uniform mix: 200,000 pairs of 10-60 px shapes (16-120 vertices) on 16384^2 tiles",
    1: "small: 1,000 pairs of <=32 px shapes (8-40 vertices) on a 4096^2 tile",
}

# Algorithmic integer work of the persistent kernel, in int32 lane-ops per
# counted unit (the counters come from an instrumented call):
#   leaf_edge_updates:    one band edge of a leaf tile XORed into its column
#                         slot: a 64-bit XOR -> 2
#   leaf_staging_edges:   one ring edge tested for a tile's band: vertical
#                         test, span clip (4), X test (2), keep (2), slot (1),
#                         row mask (2) -> 12
#   classify_edge_visits: one ring edge against a split grid: hover test and
#                         cell masks (12), first-pixel parity range and masks (12)
#   ring_scan_vertices:   one vertex of a pair's rings: extent (4 min/max),
#                         shoelace term (2 multiplies and a subtract in 64 bits: 6)
#   union_tile_vertices:  one vertex of a pair counted on one leaf tile: union
#                         extent only (4 min/max)
#   leaf_boxes:           one leaf tile: per ring a 64-bit prefix XOR over the
#                         64 column lanes (6 steps x 2 words), then the AND and
#                         popcount of both masks -> (2 x 12 + 2) x 64
#   leaf_vertex_updates:  one ring vertex XORed into its column slot by the
#                         union tile's vertex form (each vertical edge's two
#                         end points together stand for one edge update) -> 1
ALGO_OPS = {
    "leaf_edge_updates": 2,
    "leaf_vertex_updates": 1,
    "leaf_staging_edges": 12,
    "classify_edge_visits": 24,
    "ring_scan_vertices": 10,
    "union_tile_vertices": 4,
    "leaf_boxes": 26 * 64,
}
# int32 VALU peak of MI355X, lane-operations per second: the fp32 vector peak
# of 157.3 TFLOP/s counts an FMA as two flops, so the vector units retire
# 78.6 T lane-instructions/s (128 lanes per CU per clock at 2.4 GHz), and a
# plain 32-bit integer add or XOR issues at that rate (the device's own
# add/xor microbenchmark sustains about 59 T, well above the 64-lane figure)
VALU_PEAK_OPS = 256 * 128 * 2.4e9
HBM_PEAK = 8.0e12


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# The translation unit of the persistent kernel: its source, the headers it
# includes, and the compiler flags.  Counters taken on another version of any
# of these are not reported.  Comments and spacing are left out of the hash,
# so that editing documentation does not void counters of the same code.
KERNEL_SOURCES = ("paper_1208_0277_amd/csrc/k_batched.hip", "paper_1208_0277_amd/csrc/sccg_device.h",
                  "paper_1208_0277_amd/csrc/sccg_common.h", "include/sccg.h")


def _code_only(text: str) -> str:
    import re
    out, i, n = [], 0, len(text)
    while i < n:
        if text.startswith("//", i):
            i = text.find("\n", i)
            i = n if i < 0 else i
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif text[i] in "\"'":
            q, j = text[i], i + 1
            while j < n and text[j] != q:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(text[i])
            i += 1
    return re.sub(r"\s+", " ", "".join(out)).strip()


def kernel_source_hash() -> str:
    from paper_1208_0277_amd import build as _build
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    h.update(" ".join(_build.FLAGS).encode())
    return h.hexdigest()[:16]


#: offered load of the serving summary's saturated run (jobs/s)
SATURATED_RATE = 2000.0

#: the calibration sample of the autotuner is drawn with the timed
#: workload's seed plus this offset
CALIBRATION_SEED_OFFSET = 1_000_003

PROFILE_STEMS = {3: "k_batch_call_heavy_tailed_2M", 4: "k_batch_call_set_level_64_tiles"}


def tail_summary(wt):
    """Load balance of one kernel from its waves' (start, end) stamps (100 MHz
    counter): the span from the first start to the last end, the median
    wave's end, and the tail fraction (last end - median end) / span."""
    if len(wt) == 0:
        return None
    t0 = int(wt[:, 0].min())
    ends = wt[:, 1].astype(np.float64) - t0
    span = float(ends.max())
    med = float(np.median(ends))
    return {"waves": int(len(wt)), "span_us": span / 100.0, "median_end_us": med / 100.0,
            "tail_frac": (span - med) / span if span > 0 else 0.0}


def profile_summary(workload: int, params: dict):
    """The committed counter summary of the batched kernels on this workload
    (profiles/<stem>.json), or None when it is missing, was taken on another
    version of the kernel source, or with other tuning parameters than
    `params` (None: any parameters)."""
    stem = PROFILE_STEMS.get(workload)
    if stem is None:
        return None
    path = os.path.join(ROOT, "profiles", stem + ".json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    if params is not None and \
            {k: int(v) for k, v in (d.get("params") or {}).items()} != {k: int(v) for k, v in params.items()}:
        return None
    return d


def union_box_areas(wl, sel):
    """Pixels of the bounding box of MBR(p) and MBR(q) for the pairs `sel`:
    the pixel centres the oracle classifies, against both polygons."""
    lo = np.full((len(sel), 2), np.iinfo(np.int64).max)
    hi = np.full((len(sel), 2), np.iinfo(np.int64).min)
    for P, idx in ((wl.A, wl.pa[sel]), (wl.B, wl.pb[sel])):
        starts, ends = P.off[idx], P.off[idx + 1]
        lens = ends - starts
        keep = lens > 0
        if not keep.any():
            continue
        s0, ln = starts[keep], lens[keep]
        first = np.concatenate([[0], np.cumsum(ln)[:-1]])
        pts = np.repeat(s0 - first, ln) + np.arange(int(ln.sum()))
        for d in (0, 1):
            v = P.xy[pts, d].astype(np.int64)
            lo[keep, d] = np.minimum(lo[keep, d], np.minimum.reduceat(v, first))
            hi[keep, d] = np.maximum(hi[keep, d], np.maximum.reduceat(v, first))
    w, h = hi[:, 0] - lo[:, 0], hi[:, 1] - lo[:, 1]
    return np.where((w > 0) & (h > 0), w * h, 0)


def cpu_baseline(wl, I_gpu, U_gpu, seconds: float, seed: int):
    """The oracle (row-bucketed form, all host threads up to 16) on a bounded
    random sample of the same pairs; also checks the GPU counts of that
    sample.  Rates are wall-clock rates of the whole thread pool.  A
    pixel-centre test is one pixel of the bounding box of both MBRs
    classified against one polygon (the oracle classifies every such pixel
    against both).  The pure form (every edge per pixel) is timed beside the
    row-bucketed one on the 1,000-pair small workload."""
    import oracle
    import sccg_gen
    threads = min(os.cpu_count() or 1, 16)
    rng = np.random.default_rng(seed)
    order = rng.permutation(wl.n_pairs)
    done, t_total, pos, exact, tests = 0, 0.0, 0, True, 0
    chunk = 20000
    while t_total < seconds and pos < wl.n_pairs:
        sel = np.sort(order[pos:pos + chunk])
        pos += chunk
        t = time.perf_counter()
        eI, eU = oracle.area_pairs(wl.A, wl.B, wl.pa[sel], wl.pb[sel], form=oracle.ROWS, threads=threads)
        t_total += time.perf_counter() - t
        done += len(sel)
        tests += 2 * int(union_box_areas(wl, sel).sum())
        if not (np.array_equal(eI, I_gpu[sel]) and np.array_equal(eU, U_gpu[sel])):
            exact = False
    # one thread on a fixed 1% subset (every 100th pair)
    sub = np.arange(0, wl.n_pairs, 100)
    t = time.perf_counter()
    oracle.area_pairs(wl.A, wl.B, wl.pa[sub], wl.pb[sub], form=oracle.ROWS, threads=1)
    one = len(sub) / (time.perf_counter() - t)
    # both forms on the small workload (the pure form is the plain definition)
    small = sccg_gen.pairs(1)
    forms = {}
    for name, form in (("pure", oracle.PURE), ("rows", oracle.ROWS)):
        t = time.perf_counter()
        oracle.area_pairs(small.A, small.B, small.pa, small.pb, form=form, threads=threads)
        forms[name] = small.n_pairs / (time.perf_counter() - t)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": done / t_total, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} pairs drawn uniformly (seed {seed}) from the same workload, row-bucketed "
                      f"oracle form, {t_total:.2f} s wall time on {threads} threads",
            "pixel_tests_per_s": tests / t_total, "wall_s": t_total,
            "one_core_pairs_per_s": one, "one_core_sample": f"every 100th pair ({len(sub)} pairs), 1 thread",
            "small_workload_pairs_per_s": forms,
            "nproc": os.cpu_count(), "cpu_model": model}, exact, done


def run_serving(rates, jobs, cpu_threads=0, cpu_max_pairs=0):
    """Continuous-batching server under Poisson arrivals; latency is submit
    to results on the host (the server's clock).  Every job is checked
    against the oracle's counts of the corpus.  Returns (per-rate records,
    all bit-exact, corpus pairs)."""
    import threading

    import torch

    import oracle
    import paper_1208_0277_amd as sccg
    import sccg_gen

    corpus_n = 500_000
    t0 = time.perf_counter()
    wl = sccg_gen.pairs(2, corpus_n, seed=sccg_gen.BASE_SEED + 5)
    a_xy = torch.empty(wl.A.xy.size, dtype=torch.int32, pin_memory=True).numpy()
    b_xy = torch.empty(wl.B.xy.size, dtype=torch.int32, pin_memory=True).numpy()
    a_xy[:] = wl.A.xy.reshape(-1)
    b_xy[:] = wl.B.xy.reshape(-1)
    eI, eU = oracle.area_pairs(wl.A, wl.B, wl.pa, wl.pb, form=oracle.ROWS, threads=min(os.cpu_count() or 1, 16))
    log(f"corpus: {corpus_n} pairs, {len(wl.A.xy) + len(wl.B.xy)} vertices (pinned), oracle counts in "
        f"{time.perf_counter() - t0:.1f} s")
    local = np.arange(5 * 10 ** 5, dtype=np.int32)
    srv = sccg.Server(0, cpu_threads=cpu_threads, cpu_max_pairs=cpu_max_pairs)
    rng = np.random.default_rng(sccg_gen.BASE_SEED + 5)
    out_rates, all_exact = [], True
    try:
        # warm-up: one job through every stage
        srv.submit(wl.A.off[:1001], a_xy, wl.B.off[:1001], b_xy, local[:1000], local[:1000])
        if not srv.poll(1, timeout=60.0):
            raise RuntimeError("warm-up job did not finish")
        for lam in rates:
            n_jobs = jobs
            sizes = np.exp(rng.uniform(math.log(1e3), math.log(5e5), n_jobs)).astype(np.int64)
            starts = rng.integers(0, corpus_n - sizes + 1)
            arrive = np.cumsum(rng.exponential(1.0 / lam, n_jobs))  # rate inf: all at once
            outs, errors = {}, []
            lock = threading.Lock()

            def submitter():
                t_start = time.perf_counter()
                for k in range(n_jobs):
                    delay = t_start + arrive[k] - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                    s, n = int(starts[k]), int(sizes[k])
                    oi, ou = np.empty(n, np.int64), np.empty(n, np.int64)
                    with lock:  # the job may finish before submit returns
                        try:
                            j = srv.submit(wl.A.off[s:s + n + 1], a_xy, wl.B.off[s:s + n + 1], b_xy, local[:n],
                                           local[:n], out_inter=oi, out_union=ou)
                        except Exception as e:  # reported after the run
                            errors.append(repr(e))
                            return
                        outs[j] = (k, oi, ou)

            th = threading.Thread(target=submitter)
            st0 = srv.stats()
            th.start()
            results, exact = {}, True
            deadline = time.perf_counter() + arrive[-1] + 120.0
            while len(results) < n_jobs and time.perf_counter() < deadline and not errors:
                for r in srv.poll(256, timeout=1.0):
                    with lock:
                        k, oi, ou = outs.pop(r["job_id"])
                    s, n = int(starts[k]), int(sizes[k])
                    if r["status"] != 0 or not (np.array_equal(oi, eI[s:s + n]) and np.array_equal(ou, eU[s:s + n])):
                        exact = False
                    results[k] = r
            th.join()
            if errors or len(results) < n_jobs:
                raise RuntimeError(f"rate {lam}: {len(results)} of {n_jobs} jobs finished; errors {errors[:3]}")
            # set sums against the oracle (after the run: not on the serving path)
            for k, r in results.items():
                s, n = int(starts[k]), int(sizes[k])
                si, su, nn, jj, jp = oracle.jaccard_sets(np.array([0, n], np.int64), eI[s:s + n], eU[s:s + n])
                if (r["sum_i"], r["sum_u"], r["n_contrib"], r["j"], r["jprime"]) != \
                        (int(si[0]), int(su[0]), int(nn[0]), float(jj[0]), float(jp[0])):
                    exact = False
            all_exact &= exact
            st1 = srv.stats()
            meas = [results[k] for k in range(20, n_jobs)] if n_jobs > 40 else list(results.values())
            lat = np.array([r["t_done"] - r["t_submit"] for r in meas]) * 1e3
            span = max(r["t_done"] for r in meas) - min(r["t_submit"] for r in meas)
            pairs = sum(r["n_pairs"] for r in meas)
            rec = {"rate_jobs_per_s": lam, "jobs": n_jobs, "measured_jobs": len(meas),
                   "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                   "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
                   "pairs_per_s": pairs / span,
                   "offered_pairs_per_s": float(sizes.mean() * lam) if math.isfinite(lam) else None,
                   "launches": st1["launches"] - st0["launches"], "max_jobs_per_launch": st1["max_jobs_per_launch"],
                   "admission_waits": st1["admission_waits"] - st0["admission_waits"],
                   "jobs_migrated": st1["jobs_migrated"] - st0["jobs_migrated"],
                   "pairs_migrated": st1["pairs_migrated"] - st0["pairs_migrated"], "bit_exact": bool(exact)}
            log(f"rate {lam:g}/s: p50 {rec['p50_ms']:.2f} ms, p99 {rec['p99_ms']:.2f} ms, "
                f"{rec['pairs_per_s'] / 1e6:.2f} Mpairs/s served, {rec['launches']} launches, "
                f"{rec['jobs_migrated']} jobs migrated, exact {exact}")
            out_rates.append(rec)
    finally:
        srv.close()
    return out_rates, bool(all_exact), corpus_n


def serve_bench(args):
    rates = [float(r) for r in args.rates.split(",")]
    out_rates, all_exact, corpus_n = run_serving(rates, args.jobs, args.cpu_threads, args.cpu_max_pairs)
    top = out_rates[-1]
    out = {
        "metric": METRIC, "value": top["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
        "steps": args.jobs, "warmup": 20, "ms_per_step": top["mean_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": WORKLOADS[5], "corpus_pairs": corpus_n,
                   "rates": [r if math.isfinite(r) else "all at once" for r in rates],
                   "cpu_threads": args.cpu_threads, "cpu_max_pairs": args.cpu_max_pairs,
                   "parallelism": "none (1 GPU)"},
        "serving": out_rates, "bit_exact_oracle_sample": bool(all_exact), "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def run_fig8(steps, warmup, autotuned=True):
    """Section 5.2's comparison (Figure 8) on a synthetic stand-in for its
    15,724-pair set: the same pairs with every coordinate multiplied by k.
    Every variant must give identical counts, and counts at k must be k^2
    times those at 1.  Returns (rows of ms per call, all exact, pairs)."""
    import torch

    import paper_1208_0277_amd as sccg
    import sccg_gen
    from paper_1208_0277_amd import autotune

    base = sccg_gen.pairs(2, 15724, seed=sccg_gen.BASE_SEED + 6)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    # PixelBox and NoSep classify every split (min_classify_cells 1) and
    # PixelBox derives every union from the areas, as the paper's design
    # does; "PixelBox, tuned" lets the autotuner skip the classification of
    # leaf-level splits of a few tiles and counts pairs that fit one leaf
    # tile directly there
    variants = [("PixelOnly", sccg.SCCG_BATCHED, {"flags": sccg.SCCG_F_PIXEL_ONLY}),
                ("PixelBox-NoSep", sccg.SCCG_BATCHED, {"flags": sccg.SCCG_F_NO_SEP, "min_classify_cells": 1}),
                ("PixelBox", sccg.SCCG_BATCHED, {"min_classify_cells": 1, "flags": sccg.SCCG_F_NO_UNION_TILE}),
                ("PixelBox, tuned", sccg.SCCG_BATCHED, {}),
                ("Algorithm 1 (plain)", sccg.SCCG_PLAIN, {})]
    rows, exact, ref1 = [], True, None
    for k in range(1, 6):
        dA = sccg.DevicePolys.from_host(base.A.off, base.A.xy * k, dev)
        dB = sccg.DevicePolys.from_host(base.B.off, base.B.xy * k, dev)
        pa = torch.from_numpy(base.pa).to(dev)
        pb = torch.from_numpy(base.pb).to(dev)
        I = torch.empty(base.n_pairs, dtype=torch.int64, device=dev)
        U = torch.empty_like(I)
        rec, ref = {"k": k}, None
        for name, mode, fixed in variants:
            ctx = sccg.Context(0, stream=stream, **fixed)
            with torch.cuda.stream(stream):
                tuned = {}
                if autotuned:
                    tuned = autotune.tune(ctx, dA, dB, pa, pb, I, U, mode=mode, workload_key=f"fig8/{name}/{k}",
                                          steps=2, use_cache=False, log=lambda m: None)
                    ctx.set_params(**{**tuned, **fixed})
                for _ in range(warmup):
                    ctx.area_pairs(dA, dB, pa, pb, out_inter=I, out_union=U, mode=mode)
                ctx.sync()
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(steps):
                    ctx.area_pairs(dA, dB, pa, pb, out_inter=I, out_union=U, mode=mode)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t) * 1e3 / steps
                ctx.sync()
            got = (I.cpu().numpy(), U.cpu().numpy())
            ctx.close()
            if ref is None:
                ref = got
            exact &= bool(np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1]))
            rec[name + "_ms"] = ms
            log(f"k={k} {name}: {ms:.3f} ms ({base.n_pairs / (ms / 1e3) / 1e6:.1f} Mpairs/s)")
        if ref1 is None:
            ref1 = ref
        exact &= bool(np.array_equal(ref[0], k * k * ref1[0]) and np.array_equal(ref[1], k * k * ref1[1]))
        rows.append(rec)
    return rows, bool(exact), base.n_pairs


def fig8_bench(args):
    rows, exact, n_pairs = run_fig8(args.steps, args.warmup, not args.no_autotune)
    top = rows[-1]["PixelBox_ms"]
    out = {
        "metric": METRIC, "value": n_pairs / (top / 1e3), "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": top, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": WORKLOADS[6], "n_pairs": n_pairs, "value_at": "PixelBox, k = 5",
                   "parallelism": "none (1 GPU)"},
        "figure8": rows, "bit_exact_across_variants_and_k2": bool(exact), "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def copy_probe(mib: int, reps: int) -> int:
    """A device copy of a known byte count (each copy reads and writes `mib`
    MiB), run under the profiler to scale its HBM byte counters: FETCH_SIZE
    and WRITE_SIZE read for this copy, against the bytes it must move, give
    the factors applied to the kernel's own counter readings."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    log(f"copy probe: {reps} copies of {mib} MiB (each reads {mib} MiB and writes {mib} MiB)")
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=3, choices=[1, 2, 3, 4, 5, 6])
    ap.add_argument("--rates", type=str, default="5,20,80", help="workload 5: arrival rates (jobs/s)")
    ap.add_argument("--jobs", type=int, default=600, help="workload 5: jobs per rate")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="workload 5: host threads for jobs migrated off a full device (0 = no migration)")
    ap.add_argument("--cpu-max-pairs", type=int, default=0,
                    help="workload 5: largest job that migrates (0 = the server's default)")
    ap.add_argument("--tiles", type=int, default=64, help="workload 4: number of tiles")
    ap.add_argument("--pairs", type=int, default=None, help="override the pair count (not the headline)")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--params", type=str, default=None,
                    help='fixed batched parameters as JSON (e.g. \'{"min_queue_cells": 24}\'); skips the autotuner')
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="headline run: skip the serving summary")
    ap.add_argument("--serve-jobs", type=int, default=240, help="headline run: jobs of the serving summary")
    ap.add_argument("--no-fig8", action="store_true", help="headline run: skip the Figure 8 summary")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB --steps times (counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the pair path has no cross-GPU "
              f"exchange: it would shard by pair ranges (or whole tiles) with one all-reduce of the per-set sums.",
              file=sys.stderr)
        return 2

    if args.copy_probe:
        return copy_probe(args.copy_probe, args.steps)
    if args.workload == 5:
        return serve_bench(args)
    if args.workload == 6:
        return fig8_bench(args)

    import torch

    import paper_1208_0277_amd as sccg
    import sccg_gen
    from paper_1208_0277_amd import autotune

    t0 = time.perf_counter()
    if args.workload == 4:
        wl = sccg_gen.sets(n_tiles=args.tiles, tile_side=8192, cell=64)
        log(f"generated workload 4: {args.tiles} tiles, {wl.A.n} + {wl.B.n} polygons, {wl.n_pairs} candidate "
            f"pairs in {time.perf_counter() - t0:.1f} s")
    else:
        n_pairs = args.pairs or sccg_gen.DEFAULT_PAIRS[args.workload]
        wl = sccg_gen.pairs(args.workload, n_pairs)
        log(f"generated workload {args.workload}: {wl.n_pairs} pairs, {len(wl.A.xy) + len(wl.B.xy)} vertices, "
            f"{int(wl.blob.sum())} blobs in {time.perf_counter() - t0:.1f} s")
    with_sets = args.workload == 4

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    dA = sccg.DevicePolys.from_host(wl.A.off, wl.A.xy, dev)
    dB = sccg.DevicePolys.from_host(wl.B.off, wl.B.xy, dev)
    pa = torch.from_numpy(wl.pa).to(dev)
    pb = torch.from_numpy(wl.pb).to(dev)
    I = torch.empty(wl.n_pairs, dtype=torch.int64, device=dev)
    U = torch.empty(wl.n_pairs, dtype=torch.int64, device=dev)
    so = torch.from_numpy(wl.set_off).to(dev)
    torch.cuda.synchronize()
    ctx = sccg.Context(0, stream=stream)
    ctx.reserve(dA.n, dB.n, wl.n_pairs)
    wkey = f"w{args.workload}/{wl.n_pairs}"

    # The autotuner scores candidates on a calibration sample: the same mix
    # drawn under another seed (workload 4: a quarter of the tiles), never
    # the timed pairs.
    calib = {}
    cal_dev = None
    if not args.params and not args.no_autotune:
        t = time.perf_counter()
        cseed = wl.seed + CALIBRATION_SEED_OFFSET
        if with_sets:
            cwl = sccg_gen.sets(n_tiles=max(1, args.tiles // 4), tile_side=8192, cell=64, seed=cseed)
        else:
            cwl = sccg_gen.pairs(args.workload, wl.n_pairs, seed=cseed)
        cal_dev = (sccg.DevicePolys.from_host(cwl.A.off, cwl.A.xy, dev),
                   sccg.DevicePolys.from_host(cwl.B.off, cwl.B.xy, dev),
                   torch.from_numpy(cwl.pa).to(dev), torch.from_numpy(cwl.pb).to(dev),
                   torch.empty(cwl.n_pairs, dtype=torch.int64, device=dev),
                   torch.empty(cwl.n_pairs, dtype=torch.int64, device=dev))
        calib = {"sample": f"{WORKLOADS[args.workload].split(':')[0]}, {cwl.n_pairs} pairs, seed {cseed} "
                           f"(the timed pairs use seed {wl.seed})", "seed": cseed, "n_pairs": cwl.n_pairs}
        torch.cuda.synchronize()
        log(f"calibration sample: {cwl.n_pairs} pairs, seed {cseed} ({time.perf_counter() - t:.1f} s)")

    with torch.cuda.stream(stream):
        tuned = {}
        if args.params:
            tuned = json.loads(args.params)
            ctx.set_params(**tuned)
            log(f"fixed batched parameters {tuned}")
        elif not args.no_autotune:
            t = time.perf_counter()
            ctx.reserve(max(dA.n, cal_dev[0].n), max(dB.n, cal_dev[1].n), max(wl.n_pairs, calib["n_pairs"]))
            # the descent starts from the committed profile's parameters when
            # that profile was taken on this kernel source
            prof0 = profile_summary(args.workload, None)
            start = prof0["params"] if prof0 else None
            tuned = autotune.tune(ctx, *cal_dev, mode=sccg.SCCG_BATCHED, workload_key=wkey, use_cache=False,
                                  log=log, start=start)
            calib["batched_params"] = tuned
            calib["start"] = start
            log(f"autotuned batched parameters {tuned} on the calibration sample in {time.perf_counter() - t:.1f} s")

        sets_out = [None]

        def step():
            ctx.area_pairs(dA, dB, pa, pb, out_inter=I, out_union=U, mode=sccg.SCCG_BATCHED)
            if with_sets:
                sets_out[0] = ctx.jaccard_sets(so, I, U)

        for _ in range(args.warmup):
            step()
        ctx.sync()
        torch.cuda.synchronize()
        # ---------------- timed region: exactly `steps` steps -----------------
        t_start = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t_end = time.perf_counter()
        # -----------------------------------------------------------------------
        ctx.sync()
        ms_per_step = (t_end - t_start) * 1e3 / args.steps
        value = wl.n_pairs / (ms_per_step / 1e3)
        gI, gU = I.cpu().numpy(), U.cpu().numpy()
        gsets = [t.cpu().numpy() if t is not None else None for t in sets_out[0]] if with_sets else None
        log(f"batched: {ms_per_step:.3f} ms/step, {value / 1e6:.1f} Mpairs/s")

        # device time of the batched call: HIP events on its stream around all of its kernels
        ctx.set_timing(True)
        for _ in range(args.steps):
            step()
        k_ms, k_n = ctx.get_timing()
        ctx.set_timing(False)
        k_avg_ms = k_ms / max(k_n, 1)
        # per-wave stamps (a call without counters: their atomics would
        # slow it), then the work counters (instrumented call); neither timed
        ctx.set_stats(False, stamps=True)
        step()
        ctx.sync()
        balance = {name: tail_summary(ctx.wave_times(k))
                   for k, name in enumerate(("union_sweep", "medium_sweep", "persistent"))}
        ctx.set_stats(True)
        step()
        ctx.sync()
        st = ctx.get_stats()
        ctx.set_stats(False)
        same = np.array_equal(I.cpu().numpy(), gI) and np.array_equal(U.cpu().numpy(), gU)

        # plain one-pair-per-workgroup kernel on the same pairs
        plain = {}
        if not args.no_plain:
            pctx = sccg.Context(0, stream=stream)
            ptuned = {}
            if cal_dev is not None:
                t = time.perf_counter()
                ptuned = autotune.tune(pctx, *cal_dev, mode=sccg.SCCG_PLAIN, workload_key=wkey, steps=1,
                                       use_cache=False, log=log)
                calib["plain_params"] = ptuned
                log(f"autotuned plain parameters {ptuned} in {time.perf_counter() - t:.1f} s")
            pctx.area_pairs(dA, dB, pa, pb, out_inter=I, out_union=U, mode=sccg.SCCG_PLAIN)
            pctx.sync()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.plain_steps):
                pctx.area_pairs(dA, dB, pa, pb, out_inter=I, out_union=U, mode=sccg.SCCG_PLAIN)
            pctx.sync()
            p_ms = (time.perf_counter() - t) * 1e3 / args.plain_steps
            p_same = np.array_equal(I.cpu().numpy(), gI) and np.array_equal(U.cpu().numpy(), gU)
            plain = {"plain_pairs_per_s": wl.n_pairs / (p_ms / 1e3), "plain_ms_per_step": p_ms,
                     "plain_params": ptuned, "plain_equals_batched": bool(p_same),
                     "batched_vs_plain": (wl.n_pairs / (ms_per_step / 1e3)) / (wl.n_pairs / (p_ms / 1e3))}
            log(f"plain: {p_ms:.1f} ms/step; batched/plain = {plain['batched_vs_plain']:.1f}x")
            pctx.close()

    # roofline of the batched call (all of its kernels, timed together with
    # HIP events on their stream)
    algo_ops = sum(ALGO_OPS[k] * st.get(k, 0) for k in ALGO_OPS)
    achieved = algo_ops / (k_avg_ms / 1e3)
    algo_bytes = 8 * wl.n_pairs + 32 * wl.n_pairs + 8 * (len(wl.A.xy) + len(wl.B.xy)) + 16 * wl.n_pairs
    prof = profile_summary(args.workload, tuned)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s",
                "frac": achieved / VALU_PEAK_OPS, "traffic": prof["bytes_per_launch"] if prof else None,
                "kernel": "batched call: k_batch_clear_*, k_batch_setup, k_batch_sweep, "
                          "k_batch_medium, k_batch_run (one HIP event bracket)", "kernel_ms": k_avg_ms,
                "algorithmic_ops_per_launch": algo_ops, "algorithmic_bytes_per_launch": algo_bytes,
                "hbm_frac_algorithmic": (algo_bytes / (k_avg_ms / 1e3)) / HBM_PEAK}
    # the sustained integer VALU rate of this device (every lane of every
    # compute unit issuing independent adds and XORs)
    try:
        sustained, _ = ctx.valu_peak()
        roofline["peak_sustained"] = sustained / 1e12
        roofline["frac_sustained"] = achieved / sustained
        log(f"valu peak: {sustained / 1e12:.1f} T lane-ops/s sustained (nominal {VALU_PEAK_OPS / 1e12:.1f})")
    except Exception as e:  # reported, not fatal
        log(f"valu peak probe failed: {e}")
    if prof and prof.get("sq_insts_valu"):
        # counter view: every issued VALU instruction at 64 lanes, over the
        # profiled kernel time, against the same peak
        roofline["valu_issue_frac_counters"] = prof["sq_insts_valu"] * 64 / (prof["kernel_ms"] / 1e3) / VALU_PEAK_OPS
        roofline["profile"] = f"profiles/{PROFILE_STEMS[args.workload]}.md"
        # the further counter figures of the same summary, where it has them
        for key in ("valu_busy_pct", "valu_utilization_pct", "valu_int32_share", "lds_bank_conflict_pct",
                    "valu_insts_per_pixel_test", "kernels_ms"):
            if key in prof:
                roofline[key] = prof[key]

    cpu, exact_sample, n_sample = (None, None, 0)
    sets_info = {}
    if not args.no_cpu:
        cpu, exact_sample, n_sample = cpu_baseline(wl, gI, gU, args.cpu_seconds, seed=1234)
        log(f"cpu oracle: {cpu['value']:.0f} pairs/s on {n_sample} pairs, bit-exact sample: {exact_sample}")
        if with_sets and n_sample == wl.n_pairs:
            import oracle
            eI, eU = oracle.area_pairs(wl.A, wl.B, wl.pa, wl.pb, form=oracle.ROWS)
            osi, osu, onn, oj, ojp = oracle.jaccard_sets(wl.set_off, eI, eU)
            sets_info["sets_bit_exact"] = bool(np.array_equal(gsets[0], osi) and np.array_equal(gsets[1], osu) and
                                               np.array_equal(gsets[3], oj) and np.array_equal(gsets[4], ojp))
    if with_sets:
        # the filter stage on the device too: join, pair counts and set sums
        with torch.cuda.stream(stream):
            dao = torch.from_numpy(wl.a_set_off).to(dev)
            dbo = torch.from_numpy(wl.b_set_off).to(dev)
            jctx = sccg.Context(0, stream=stream, **tuned)
            jpa, jpb, jso = jctx.join_sets(dA, dB, dao, dbo)
            jctx.sync()
            same_join = bool(np.array_equal(jpa.cpu().numpy(), wl.pa) and np.array_equal(jpb.cpu().numpy(), wl.pb)
                             and np.array_equal(jso.cpu().numpy(), wl.set_off))
            reps = max(1, args.steps // 4)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                jctx.join_sets(dA, dB, dao, dbo, cap=wl.n_pairs)
            torch.cuda.synchronize()
            join_ms = (time.perf_counter() - t) * 1e3 / reps
            t = time.perf_counter()
            for _ in range(reps):
                jpa, jpb, jso = jctx.join_sets(dA, dB, dao, dbo, cap=wl.n_pairs)
                jI, jU = jctx.area_pairs(dA, dB, jpa, jpb, mode=sccg.SCCG_BATCHED)
                jctx.jaccard_sets(jso, jI, jU)
            torch.cuda.synchronize()
            e2e_ms = (time.perf_counter() - t) * 1e3 / reps
            jctx.sync()
            jctx.close()
        log(f"device join: {join_ms:.3f} ms, equals the host join: {same_join}; join + pairs + sets: {e2e_ms:.3f} ms")
        sets_info["device_join"] = {"join_ms": join_ms, "equals_host_join": same_join,
                                    "end_to_end_ms": e2e_ms, "end_to_end_pairs_per_s": wl.n_pairs / (e2e_ms / 1e3)}
        sets_info.update({"n_sets": int(len(wl.set_off) - 1), "J_mean": float(np.mean(gsets[3])),
                          "J_min": float(np.min(gsets[3])), "J_max": float(np.max(gsets[3])),
                          "Jprime_mean": float(np.mean(gsets[4]))})

    # the serving loop and the Figure 8 comparison, summarized beside the
    # headline (after its timed region)
    extras = {}
    if args.workload == 3 and not args.no_serving:
        # 80 jobs/s, then an offered load above what the device takes in
        # (jobs queue for admission and launches merge them)
        recs, sexact, corpus_n = run_serving([80.0, SATURATED_RATE], args.serve_jobs)
        r, q = recs
        extras["serving"] = {"workload": WORKLOADS[5].replace(
                                 "5, 20 and 80 jobs/s, 600 jobs per rate",
                                 f"80 and {SATURATED_RATE:g} jobs/s, {args.serve_jobs} jobs per rate"),
                             "rate_jobs_per_s": 80.0, "jobs": r["jobs"], "measured_jobs": r["measured_jobs"],
                             "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"], "pairs_per_s": r["pairs_per_s"],
                             "offered_pairs_per_s": r["offered_pairs_per_s"], "launches": r["launches"],
                             "max_jobs_per_launch": r["max_jobs_per_launch"],
                             "saturated": {"rate_jobs_per_s": SATURATED_RATE, "jobs": q["jobs"],
                                           "p50_ms": q["p50_ms"], "p99_ms": q["p99_ms"],
                                           "pairs_per_s": q["pairs_per_s"],
                                           "offered_pairs_per_s": q["offered_pairs_per_s"],
                                           "launches": q["launches"],
                                           "mean_jobs_per_launch": q["jobs"] / max(q["launches"], 1),
                                           "max_jobs_per_launch": q["max_jobs_per_launch"],
                                           "admission_waits": q["admission_waits"]},
                             "bit_exact": sexact}
    if args.workload == 3 and not args.no_fig8:
        rows, fexact, n8 = run_fig8(steps=5, warmup=1)
        extras["figure8"] = {"workload": WORKLOADS[6], "pairs": n8, "ms_per_call": rows,
                             "bit_exact_across_variants_and_k2": fexact}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "n_pairs": wl.n_pairs, "seed": wl.seed,
                   "n_tiles": args.tiles if with_sets else None,
                   "mode": "batched", "params": tuned, "parallelism": "none (1 GPU)"},
        "pixel_tests_per_s": st["leaf_pixel_tests"] / (ms_per_step / 1e3),
        "covered_pixels_per_s": st["covered_pixels"] / (ms_per_step / 1e3),
        **plain,
        "bit_exact_oracle_sample": exact_sample,
        "oracle_sample_pairs": n_sample,
        "repeat_identical": bool(same),
        **sets_info,
        "autotune": calib or None,
        "load_balance": balance,
        "stats": st,
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
