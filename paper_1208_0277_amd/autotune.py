"""Autotuner for the tuning parameters of both modes.

Coordinate descent over a small candidate grid: each parameter is swept in
turn with the others held at the best values found so far; a candidate is
scored by pairs/s over a few timed calls on the caller's workload and
replaces the best only when it is faster by more than MARGIN.  Every
candidate must reproduce the first candidate's counts bit for bit (no tuning
parameter may change a result); a candidate that does not is an error.
Results are cached in JSON, keyed by GPU architecture, CU count, mode and a
workload key supplied by the caller.
"""

from __future__ import annotations

import hashlib
import json
import os
import time

import paper_1208_0277_amd as sccg

#: batched-mode candidates, swept in this order
BATCHED_SPACE = [
    ("min_queue_cells", [24, 8, 65]),
    ("queue_chunk", [16, 8, 32, 64]),
    ("waves_per_wg", [4, 2, 8]),
    ("heavy_verts", [512, 1024, 2048]),
    ("min_classify_cells", [26, 1, 10, 65]),
    ("sweep_pair_box", [1, 2]),
]

#: plain-mode candidates: the pixelization threshold T (Section 3.4 puts the
#: best T between n^2/8 and n^2 for n threads per block) and the block size
PLAIN_SPACE = [
    ("box_threshold", [2048, 512, 1024, 4096]),
    ("wg_size", [64, 128]),
]

#: fraction by which a candidate must beat the best so far to replace it
MARGIN = 0.02

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sccg", "autotune.json")


def _digest(I, U) -> str:
    h = hashlib.sha256()
    h.update(I.cpu().numpy().tobytes())
    h.update(U.cpu().numpy().tobytes())
    return h.hexdigest()


def _device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "unknown")
    return f"{arch}/{p.multi_processor_count}"


def tune(ctx, dA, dB, pa, pb, I, U, mode=sccg.SCCG_BATCHED, workload_key="", steps=8, use_cache=True,
         space=None, log=None, start=None):
    """Return the best parameter dict for this workload and leave it set on ctx.
    `start` (optional): the values the descent starts from, e.g. an earlier
    tuning's result; each must be one of its parameter's candidates."""
    space = space or (BATCHED_SPACE if mode == sccg.SCCG_BATCHED else PLAIN_SPACE)
    key = f"{_device_key()}/{'batched' if mode == sccg.SCCG_BATCHED else 'plain'}/{workload_key}"
    cache = {}
    if use_cache and os.path.exists(CACHE):
        try:
            with open(CACHE) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        best = cache[key]["params"]
        p = dict(ctx.get_params())
        p.update(best)
        ctx.set_params(**p)
        return best
    base = dict(ctx.get_params())
    if any(name == "wg_size" for name, _ in space):
        base["split_gx"] = base["split_gy"] = 0  # the split grid follows the block size
    best = {name: vals[0] for name, vals in space}
    for name, vals in space:
        if start and name in start and int(start[name]) in vals:
            best[name] = int(start[name])
    call_args = (dA, dB, pa, pb)
    ref = None
    scores = {}

    def score(params):
        k = json.dumps(params, sort_keys=True)
        if k in scores:
            return scores[k]
        p = dict(base)
        p.update(params)
        ctx.set_params(**p)
        dt = _timed(ctx, call_args, I, U, mode, steps)
        nonlocal ref
        d = _digest(I, U)
        if ref is None:
            ref = d
        elif d != ref:
            raise RuntimeError(f"tuning parameters {params} changed the counts")
        scores[k] = dt
        if log:
            log(f"autotune {params}: {dt * 1e3:.3f} ms")
        return dt

    best_t = score(best)
    for name, vals in space:
        for v in vals:
            if v == best[name]:
                continue
            cand = dict(best)
            cand[name] = v
            t = score(cand)
            # a candidate must win by more than timing noise, so that
            # repeated tunings of one workload settle on the same values
            if t < best_t * (1.0 - MARGIN):
                best, best_t = cand, t
    p = dict(base)
    p.update(best)
    ctx.set_params(**p)
    if use_cache:
        cache[key] = {"params": best, "ms": best_t * 1e3}
        try:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            with open(CACHE, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return best


def _timed(ctx, call_args, I, U, mode, steps):
    import torch
    dA, dB, pa, pb = call_args
    ctx.area_pairs(dA, dB, pa, pb, out_inter=I, out_union=U, mode=mode)
    ctx.sync()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        ctx.area_pairs(dA, dB, pa, pb, out_inter=I, out_union=U, mode=mode)
    ctx.sync()
    return (time.perf_counter() - t) / steps
