"""Tile autotuner for batched solves.

The persistent batch kernel splits every instance into workgroup tiles of at
most `tile_cap` nonzeros, with one cap per instance size class
(pmp_batch_options).  Small caps give more, smaller tiles (better balance
across workgroups when instances are small and stop at different times);
large caps give fewer, longer tiles (more gathers in flight per workgroup).
The tuner times a fixed number of batch iterations for each candidate cap,
one size class at a time (the other classes held at their current best), and
keeps the fastest; it then picks the number of resident workgroups per CU
of the persistent grid (more hide latency, fewer make the grid barriers
cheaper).  When some instance has congested links (Section V-C: link rows of
more than 4096 nonzeros), a heavy-row class follows: the chunk of nonzeros
that one workgroup sums of such a row (pmp_batch_options.heavy_chunk; small
chunks spread a row over more workgroups, large ones save the second-stage
adds).  FP32 instances with a finite box sum these rows in fixed point, so
there the chunk changes only the time; FP64 sums move in their last bits.
Results are cached per GPU architecture and class in a JSON file.
"""
from __future__ import annotations

import json
import os
import time

CANDIDATES = (1024, 2048, 4096, 8192)
GRID_CANDIDATES = (1, 2, 4, 8)          # resident workgroups per CU
HEAVY_CANDIDATES = (1024, 2048, 4096, 8192, 16384, 65536)   # nonzeros per chunk of a long row
CLASS_NAMES = ("small", "medium", "large")
LONG_ROW = 4096                         # rows longer than this are chunked


def has_heavy_rows(inst):
    """Whether some link row of the instance is longer than LONG_ROW."""
    import numpy as np
    rp = np.asarray(inst.row_ptr)
    return rp.size > 1 and int(np.diff(rp).max()) > LONG_ROW


def default_cache_path():
    return os.environ.get("PMP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pmp_mi355x",
                                       "batch_tiles.json"))


def _arch(torch):
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def load_cache(path=None):
    path = path or default_cache_path()
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def cached_options(torch, path=None):
    """pmp_batch_options from the cache for this GPU (defaults where absent)."""
    from .pmp import batch_options_default
    o = batch_options_default()
    cache = load_cache(path)
    arch = _arch(torch)
    for c, name in enumerate(CLASS_NAMES):
        key = f"{arch}:{name}"
        if key in cache:
            o.tile_cap[c] = int(cache[key]["tile_cap"])
    if f"{arch}:grid" in cache:
        o.wg_per_cu = int(cache[f"{arch}:grid"]["wg_per_cu"])
    if f"{arch}:heavy" in cache:
        o.heavy_chunk = int(cache[f"{arch}:heavy"]["heavy_chunk"])
    return o


def _time_batch(insts, dtype, options, iters, reps, **kw):
    import torch

    from .pmp import BatchSolver
    b = BatchSolver(insts, dtype=dtype, options=options, eps_abs=0.0, **kw)
    b.solve(max(2, iters // 4))                       # warm-up (graph capture)
    best = float("inf")
    for _ in range(reps):
        b.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.solve(iters)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    b.close()
    return best


def tune_batch(insts, dtype=None, iters=60, reps=2, candidates=CANDIDATES, path=None,
               log=None, heavy_candidates=HEAVY_CANDIDATES, **kw):
    """Choose tile caps per size class, the persistent grid and (with
    congested links present) the long-row chunk for these instances; update
    the cache and return (options, timings)."""
    import torch

    from .pmp import batch_options_default
    dtype = dtype or torch.float32
    opts = batch_options_default()
    present = set()
    for inst in insts:
        present.add(0 if inst.m < opts.class_m[0] else (1 if inst.m < opts.class_m[1] else 2))
    timings = {}
    for c in sorted(present):
        best_cap, best_t = opts.tile_cap[c], None
        for cap in candidates:
            opts.tile_cap[c] = cap
            t = _time_batch(insts, dtype, opts, iters, reps, **kw)
            timings[f"{CLASS_NAMES[c]}:{cap}"] = t
            if log:
                log(f"[tune] class {CLASS_NAMES[c]} cap {cap}: {t * 1e3:.2f} ms / {iters} it")
            if best_t is None or t < best_t:
                best_cap, best_t = cap, t
        opts.tile_cap[c] = best_cap
    best_g, best_t = opts.wg_per_cu, None
    for g in GRID_CANDIDATES:
        opts.wg_per_cu = g
        t = _time_batch(insts, dtype, opts, iters, reps, **kw)
        timings[f"grid:{g}"] = t
        if log:
            log(f"[tune] {g} workgroups per CU: {t * 1e3:.2f} ms / {iters} it")
        if best_t is None or t < best_t:
            best_g, best_t = g, t
    opts.wg_per_cu = best_g
    heavy = any(has_heavy_rows(i) for i in insts)
    if heavy:
        best_h, best_t = opts.heavy_chunk, None
        for h in heavy_candidates:
            opts.heavy_chunk = h
            t = _time_batch(insts, dtype, opts, iters, reps, **kw)
            timings[f"heavy:{h}"] = t
            if log:
                log(f"[tune] long-row chunk {h}: {t * 1e3:.2f} ms / {iters} it")
            if best_t is None or t < best_t:
                best_h, best_t = h, t
        opts.heavy_chunk = best_h
    path = path or default_cache_path()
    cache = load_cache(path)
    arch = _arch(torch)
    for c in sorted(present):
        cache[f"{arch}:{CLASS_NAMES[c]}"] = {"tile_cap": int(opts.tile_cap[c])}
    cache[f"{arch}:grid"] = {"wg_per_cu": int(opts.wg_per_cu)}
    if heavy:
        cache[f"{arch}:heavy"] = {"heavy_chunk": int(opts.heavy_chunk)}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return opts, timings
