#!/usr/bin/env python3
"""PMP throughput on one MI355X: iterations per second and achieved HBM
bandwidth on the large synthetic NUM instance, plus time to the 1e-4 stop
rule, with the FP64 CPU oracle timed beside it.

One step = one PMP iteration: the stream pass (CSC gather, prox, relaxation)
and the link pass (CSR gather, slack prox, averaging, dual update), with the
residual check every 10 iterations and rho balancing every 50, replayed as
captured graphs by pmp_solve (stop rule disabled in the timed region).  The
reported rate is the median of --repeats timed runs of --steps iterations,
each placed so that it spans a balancing iteration.

Workload "large": m = 5e6 links, n = 2e7 streams, route lengths from a
discrete power law P(L) ~ L^-2.5 on {3..40}, capacities lognormal(2, 1), all
log utilities w ~ U[0.5, 2], box [0, max c]; FP32 storage, int32 indices.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "PMP iters/sec + achieved HBM GB/s at n=2e7; time to 1e-4 rel. residual"
CSRC = os.path.join(ROOT, "paper_2509_10722_amd", "csrc")


def bytes_model(n, m, nnz):
    """Compulsory bytes per launch: every array touched once, gathered
    vectors counted once, FP32 values and int32 indices."""
    stream = 4 * (n + 1) + 4 * nnz + 4 * m + 4 * n + 8 * n + 4 * n   # col_ptr, row_idx, v, w, a r/w, x w
    link = 4 * (m + 1) + 4 * nnz + 4 * n + 4 * m + 3 * 8 * m + 4 * m  # row_ptr, col_idx, x, c, u/b/zs r/w, v w
    return {"stream": stream, "link": link, "iteration": stream + link}


def source_sha(files):
    h = hashlib.sha256()
    for fn in files:
        with open(os.path.join(CSRC, fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, layout, workload):
    """Counter-measured HBM bytes per launch from profiles/ (FETCH_SIZE and
    WRITE_SIZE, scaled by a calibration copy), if taken on the current source
    of that kernel; None otherwise."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{layout}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha") != source_sha(t.get("source_files", [])):
        return None
    return t.get("bytes_per_launch")


def calibrate_copy(log):
    """An elementwise kernel that reads and writes 1 GiB each (known bytes),
    the scale for the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"[bench] calibration: 3 x torch.mul over {src.numel() * 4} bytes in and out")
    del src, dst


def bench_batched(args, log):
    """Pattern 2: the batched transit workload (64 instances, m log-uniform
    on [1e3, 1e5], n = 5m, degraded capacities) solved to the 1e-4 rule by
    one persistent launch, against solving the instances one by one."""
    import numpy as np
    import torch

    from paper_2509_10722_amd import autotune, instances
    from paper_2509_10722_amd.pmp import BatchSolver, Solver

    if args.calibrate_copy:
        calibrate_copy(log)
    insts = [i.rounded(np.float32) for i in instances.batched(scale=args.scale)]
    tot = {"m": sum(i.m for i in insts), "n": sum(i.n for i in insts),
           "nnz": sum(i.nnz for i in insts)}
    log(f"[bench] batched: {len(insts)} instances, {tot}")
    if args.tune:
        opts, timings = autotune.tune_batch(insts, dtype=torch.float32, log=log)
    else:
        opts = autotune.cached_options(torch)
    caps = list(opts.tile_cap) + [int(opts.wg_per_cu)]

    def batched_solve(profile):
        opts.profile = int(profile)
        b = BatchSolver(insts, dtype=torch.float32, options=opts)
        b.solve(20)                     # warm-up: graph capture, first touch
        b.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = b.solve(args.tol_max_iter)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        prof = b.profile() if profile else None
        b.close()
        return t, res, prof

    tb, res, _ = batched_solve(False)
    iters = [r["iterations"] for r in res]
    conv = sum(r["converged"] for r in res)
    log(f"[bench] batched solve: {tb:.3f} s, {conv}/{len(insts)} converged, "
        f"iterations {min(iters)}..{max(iters)}")
    if args.batch_only:   # one solve and nothing else (for counter runs)
        return
    # the same solve again with the kernel's phase clocks on
    tprof, _, phases = batched_solve(True)
    log(f"[bench] phases (ms per workgroup, solve {tprof:.3f} s): {phases}")
    # the same instances one by one (graph-replayed pmp_solve each)
    tp = 0.0
    plain_iters = []
    for inst in insts:
        s = Solver(inst, dtype=torch.float32, max_iter=args.tol_max_iter)
        s.solve()
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve()
        torch.cuda.synchronize()
        tp += time.perf_counter() - t0
        plain_iters.append(r["iterations"])
        s.close()
    work = sum(bytes_model(i.n, i.m, i.nnz)["iteration"] * k for i, k in zip(insts, iters))
    line = {
        "metric": "batched PMP instance-iterations/sec (64 transit instances, to 1e-4)",
        "value": round(sum(iters) / tb, 1), "unit": "instance-iter/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched transit x{len(insts)}", **tot,
                   "tile_cap": caps[:3], "wg_per_cu": caps[3]},
        "time_s": round(tb, 4), "plain_time_s": round(tp, 4),
        "speedup_vs_plain": round(tp / tb, 3), "converged": conv,
        "iterations_equal_plain": sum(int(a == c) for a, c in zip(iters, plain_iters)),
        "iterations": {"min": int(min(iters)), "median": int(np.median(iters)),
                       "max": int(max(iters))},
        "model_gbs": round(work / tb / 1e9, 2),
        "phases_ms": {k: round(v, 2) for k, v in phases.items()},
    }
    print(json.dumps(line), flush=True)


def bench_batched_congested(args, log):
    """Pattern 2 under Section V-C's congestion: the 64 transit instances of
    the batched workload, each with 0.1% of its links added to 10% of its
    streams (the largest get rows of up to 50,000 nonzeros), iterated a fixed
    number of times (no stop rule, so every instance does the same work) by
    one persistent launch: long rows in chunk tiles of heavy_chunk nonzeros
    against one workgroup per long row, and against one-by-one solves."""
    import numpy as np
    import torch

    from paper_2509_10722_amd import autotune, instances
    from paper_2509_10722_amd.pmp import BatchSolver, Solver

    base = instances.batched(scale=args.scale)
    insts = [instances.congested(i, link_frac=args.link_frac, stream_frac=args.stream_frac,
                                 seed=100 + k).rounded(np.float32) for k, i in enumerate(base)]
    del base
    tot = {"m": sum(i.m for i in insts), "n": sum(i.n for i in insts),
           "nnz": sum(i.nnz for i in insts),
           "long_rows": int(sum(int(np.sum(np.diff(i.row_ptr) > autotune.LONG_ROW)) for i in insts)),
           "longest_row": int(max(int(np.diff(i.row_ptr).max()) for i in insts))}
    log(f"[bench] congested batch: {len(insts)} instances, {tot}")
    K = args.steps
    if args.tune:
        opts, _ = autotune.tune_batch(insts, dtype=torch.float32, log=log)
    else:
        opts = autotune.cached_options(torch)
    if args.heavy_chunk:
        opts.heavy_chunk = args.heavy_chunk

    def batched(chunk):
        """Time K iterations with long rows in chunks of `chunk` nonzeros."""
        opts.heavy_chunk = chunk
        b = BatchSolver(insts, dtype=torch.float32, options=opts, eps_abs=0.0)
        b.solve(20)
        b.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.solve(K)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        x = [b.solution(k)[0].cpu() for k in range(len(insts))]
        b.close()
        return t, x

    chunk = int(opts.heavy_chunk)
    tb, xb = batched(chunk)
    log(f"[bench] heavy_chunk {chunk}: {K} iterations in {tb:.3f} s")
    others = {}
    for c in args.chunk_sweep:
        others[c] = batched(c)[0]
        log(f"[bench] heavy_chunk {c}: {K} iterations in {others[c]:.3f} s")
    t1, x1 = batched(1 << 20)
    log(f"[bench] one workgroup per long row: {K} iterations in {t1:.3f} s")
    same = all(torch.equal(a, c) for a, c in zip(xb, x1))
    tp = 0.0
    for inst in insts:
        s = Solver(inst, dtype=torch.float32, eps_abs=0.0, max_iter=K)
        s.solve()                       # graph capture
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve()
        torch.cuda.synchronize()
        tp += time.perf_counter() - t0
        s.close()
    log(f"[bench] one by one: {tp:.3f} s")
    line = {
        "metric": "batched PMP instance-iterations/sec (64 congested transit instances, fixed K)",
        "value": round(len(insts) * K / tb, 1), "unit": "instance-iter/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"congested batched transit x{len(insts)}", **tot, "K": K,
                   "heavy_chunk": chunk, "link_frac": args.link_frac,
                   "stream_frac": args.stream_frac},
        "time_s": round(tb, 4), "row_per_workgroup_time_s": round(t1, 4),
        "chunking_speedup": round(t1 / tb, 3), "plain_time_s": round(tp, 4),
        "speedup_vs_plain": round(tp / tb, 3), "iterates_equal_across_chunks": bool(same),
        "chunk_sweep_s": {str(c): round(t, 4) for c, t in others.items()},
    }
    print(json.dumps(line), flush=True)


def bench_adjoint(args, log):
    """Pattern 3: gradient of sum_j w_j log x_j^K (K = 500, checkpoints every
    25) with respect to c and w on the adjoint workload, against K plain
    iterations."""
    import numpy as np
    import torch

    from paper_2509_10722_amd import instances
    from paper_2509_10722_amd.pmp import Solver

    inst = instances.adjoint(scale=args.scale).rounded(np.float32)
    K, s = 500, 25
    solver = Solver(inst, dtype=torch.float32, adapt_every=0)
    layout = solver.layout_in_use()
    solver.iterate(K)
    solver.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.iterate(K)
    solver.residuals()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    solver.reset()
    solver.forward_ckpt(K, s)
    solver.backward()
    solver.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = solver.forward_ckpt(K, s)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    gc, gw = solver.backward()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    solver.close()
    line = {
        "metric": "PMP reverse mode: seconds per gradient (K=500 unrolled iterations)",
        "value": round(t_fwd + t_bwd, 4), "unit": "s", "n_gpus": 1,
        "higher_is_better": False, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"adjoint (m={inst.m}, n={inst.n}, nnz={inst.nnz})", "K": K,
                   "checkpoint_every": s, "layout": layout, "rho": "fixed 1"},
        "verified": "the same configuration (FP32, binned, K=500, s=25, fixed rho) against "
                    "central differences (h=1e-3) of the FP64 oracle at scale 0.1 and 1: "
                    "tests/test_gpu_adjoint.py",
        "forward_s": round(t_fwd, 4), "backward_s": round(t_bwd, 4),
        "plain_K_iterations_s": round(t_plain, 4),
        "ratio_vs_plain": round((t_fwd + t_bwd) / t_plain, 3), "J": J,
        "grad_c_norm": float(torch.linalg.vector_norm(gc.double())),
        "grad_w_norm": float(torch.linalg.vector_norm(gw.double())),
    }
    print(json.dumps(line), flush=True)


def bench_warmstart(args, log):
    """Section V-D: re-solve after capacity degradation (25% of links lose
    50%) and after link failure (25% of links fail; pruned on the device),
    cold versus warm started from the previous solution.  Two warm starts:
    "full" keeps the whole iterate (a, b, zs, u, rho); "primal" keeps the
    stream side a and rho and restarts the link side b = zs = u = 0."""
    import numpy as np
    import torch

    from paper_2509_10722_amd import instances
    from paper_2509_10722_amd.pmp import Solver

    inst = instances.make(args.config, scale=args.scale).rounded(np.float32)
    rng = np.random.default_rng(7)
    out = {}

    def timed_solve(s):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    def primal_only(s, buf):
        b = buf.clone()
        esz = 4 if s.dtype == torch.float32 else 8
        b[s.n * esz:(s.n + 3 * s.m) * esz].zero_()
        return b

    def summary(rc, tc, warm):
        d = {"cold_iters": rc["iterations"], "cold_s": round(tc, 4)}
        for mode, (rw, tw) in warm.items():
            d[f"warm_{mode}_iters"] = rw["iterations"]
            d[f"warm_{mode}_s"] = round(tw, 4)
            d[f"speedup_{mode}"] = round(tc / tw, 3)
        return d

    rule = rule_params(args)
    base = Solver(inst, dtype=torch.float32, max_iter=args.tol_max_iter, **rule)
    r0, t_base = timed_solve(base)
    log(f"[bench] base solve: {r0['iterations']} it, {t_base:.3f} s")
    st0 = base.get_state()
    # degradation: warm = same handle with the new capacities
    c_new = (inst.c * np.where(rng.random(inst.m) < 0.25, 0.5, 1.0)).astype(np.float32)
    base.update_capacity(c_new)
    warm = {"full": timed_solve(base)}
    base.set_state(primal_only(base, st0))
    warm["primal"] = timed_solve(base)
    deg = instances.Instance(inst.name, inst.m, inst.n, inst.row_ptr, inst.col_idx,
                             c_new.astype(np.float64), inst.w, inst.utility, inst.lo, inst.hi)
    cold = Solver(deg, dtype=torch.float32, max_iter=args.tol_max_iter, **rule)
    rc, tc = timed_solve(cold)
    cold.close()
    out["degradation"] = summary(rc, tc, warm)
    log(f"[bench] degradation: {out['degradation']}")
    # failure: prune on the device (compaction, then setup of the pruned
    # instance), warm start from the base solution restricted to survivors
    base.update_capacity(inst.c.astype(np.float32))
    base.set_state(st0)
    failed = (rng.random(inst.m) < 0.25).astype(np.uint8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pw, _, _ = base.prune(failed)
    torch.cuda.synchronize()
    t_prune = time.perf_counter() - t0
    base.close()
    pr = pw.instance
    stp = pw.get_state()
    warm = {"full": timed_solve(pw)}
    pw.set_state(primal_only(pw, stp))
    warm["primal"] = timed_solve(pw)
    pw.close()
    cold = Solver(pr, dtype=torch.float32, max_iter=args.tol_max_iter, **rule)
    rc, tc = timed_solve(cold)
    cold.close()
    out["failure"] = {"links_failed": int(failed.sum()), "m_pruned": pr.m, "n_pruned": pr.n,
                      "prune_setup_s": round(t_prune, 4), **summary(rc, tc, warm),
                      "original_cold_s": round(t_base, 4),
                      "resolve_vs_original_cold": round(
                          t_base / (t_prune + min(w[1] for w in warm.values())), 3)}
    log(f"[bench] failure: {out['failure']}")
    line = {"metric": "warm-start re-solve speedup to 1e-4 (Section V-D)",
            "value": out["degradation"]["speedup_full"], "unit": "x", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{args.config} (m={inst.m}, n={inst.n}, nnz={inst.nnz})",
                       "stop_rule": args.rule, **rule},
            **out}
    print(json.dumps(line), flush=True)


def rule_params(args):
    """--rule abs: Section III-F's absolute rule, eps_abs = 1e-4; rel: its
    relative form, eps_rel = 1e-4 of max(||p||, ||z||) and ||rho u||."""
    return ({"eps_abs": 1e-4, "eps_rel": 0.0} if args.rule == "abs"
            else {"eps_abs": 0.0, "eps_rel": 1e-4})


def bench_congested(args, log):
    """Section V-C: the same network without and with congestion (0.1% of
    links each joined by 10% of the streams), solved to the 1e-4 rule."""
    import numpy as np
    import torch

    from paper_2509_10722_amd import instances
    from paper_2509_10722_amd.pmp import Solver

    base = instances.make(args.config, scale=args.scale)
    cong = instances.congested(base)
    out = {}
    chunk = 2000
    for name, inst in (("uncongested", base), ("congested", cong)):
        inst = inst.rounded(np.float32)
        s = Solver(inst, dtype=torch.float32, max_iter=chunk, **rule_params(args))
        s.iterate(20)
        s.reset()
        # solved in chunks of `chunk` iterations (one progress line each), at
        # most --tol-max-iter in all
        done, dt = 0, 0.0
        while True:
            s.update_params(max_iter=min(chunk, args.tol_max_iter - done))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = s.solve()
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
            done += r["iterations"]
            log(f"[bench] {name}: {done} iterations, r {r['r_norm']:.3e} s {r['s_norm']:.3e} "
                f"(tol {r['eps_tol']:.3e}), {dt:.2f} s")
            if r["converged"] or done >= args.tol_max_iter:
                break
        r = dict(r, iterations=done)
        deg = np.diff(inst.row_ptr)
        out[name] = {"nnz": inst.nnz, "max_link_degree": int(deg.max()),
                     "iterations": r["iterations"], "converged": r["converged"],
                     "time_s": round(dt, 4), "layout": s.layout_in_use()}
        s.close()
        log(f"[bench] {name}: {out[name]}")
    line = {"metric": "extra iterations to 1e-4 under congestion (Section V-C)",
            "value": out["congested"]["iterations"] - out["uncongested"]["iterations"],
            "unit": "iterations", "n_gpus": 1, "higher_is_better": False, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"{args.config} (m={base.m}, n={base.n}) with 0.1% of links "
                                   f"on 10% of streams", "stop_rule": args.rule,
                       **rule_params(args)}, **out}
    print(json.dumps(line), flush=True)


def bench_transit(args, log):
    """Section VI's transit seat allocation at its stated size (m = 182,784
    links, n = 19,800 streams, w = 1): time to the 1e-4 rule in FP32, then an
    FP64 solve to 1e-8 whose path prices pi = R^T lambda are checked against
    the stationarity w_j / x_j = pi_j and compared for two routes of one OD
    pair and departure."""
    import numpy as np
    import torch

    from paper_2509_10722_amd import instances
    from paper_2509_10722_amd.pmp import Solver

    inst, meta = instances.transit_case_study()
    f32 = inst.rounded(np.float32)
    s = Solver(f32, dtype=torch.float32, max_iter=args.tol_max_iter)
    s.iterate(20)
    s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = s.solve()
    torch.cuda.synchronize()
    t_tol = time.perf_counter() - t0
    s.close()
    log(f"[bench] transit FP32 to 1e-4: {r['iterations']} it, {t_tol:.4f} s")
    d = Solver(inst, dtype=torch.float64, eps_abs=1e-8, max_iter=max(args.tol_max_iter, 200000))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rd = d.solve()
    torch.cuda.synchronize()
    t_tight = time.perf_counter() - t0
    x, _, _ = d.solution()
    x = x.cpu().numpy()
    pi = d.path_prices().cpu().numpy()
    d.close()
    inner = (x > 1e-9) & (x < inst.hi * (1 - 1e-9))
    marg = inst.w[inner] / x[inner]
    stat = float(np.max(np.abs(marg - pi[inner]) / marg)) if inner.any() else 0.0
    # two routes of OD pair 0 departing at bin 0
    sel = np.flatnonzero((meta["od"] == 0) & (meta["t0"] == 0))
    pair = [{"route": int(meta["route"][j]), "links": len(meta["routes"][0][meta["route"][j]]),
             "x": round(float(x[j]), 6), "path_price": round(float(pi[j]), 6)} for j in sel]
    line = {"metric": "transit case study: time to 1e-4 (Section VI)", "value": round(t_tol, 4),
            "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"transit case study (m={inst.m}, n={inst.n}, nnz={inst.nnz})"},
            "iterations": r["iterations"], "converged": r["converged"],
            "f64_tight": {"eps_abs": 1e-8, "iterations": rd["iterations"],
                          "converged": rd["converged"], "time_s": round(t_tight, 4),
                          "max_rel_stationarity": stat, "interior_streams": int(inner.sum())},
            "od0_departure0": pair}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of --steps iterations; the median is reported")
    ap.add_argument("--config", default="large")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--kernel-iters", type=int, default=40)
    ap.add_argument("--tol-max-iter", type=int, default=20000)
    ap.add_argument("--no-tol", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--cpu-single-iters", type=int, default=1,
                    help="iterations of the single-thread oracle run (0: skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-to-tol", action="store_true",
                    help="also run the oracle to the 1e-4 stop rule (tiny and medium only)")
    ap.add_argument("--layout", default="auto", choices=["auto", "gather", "binned"])
    ap.add_argument("--pattern", default="plain",
                    choices=["plain", "batched", "adjoint", "warmstart", "congested", "transit"],
                    help="plain: the large workload (the default line); batched / adjoint: "
                         "the two training-system patterns, one JSON line each")
    ap.add_argument("--tune", action="store_true", help="batched: run the tile autotuner first")
    ap.add_argument("--rule", default="abs", choices=["abs", "rel"],
                    help="warmstart / congested: stop rule (abs: eps_abs = 1e-4; rel: "
                         "eps_rel = 1e-4)")
    ap.add_argument("--congested", action="store_true",
                    help="batched: congested transit instances (Section V-C), fixed iterations")
    ap.add_argument("--link-frac", type=float, default=0.001,
                    help="batched --congested: fraction of each instance's links made hot")
    ap.add_argument("--stream-frac", type=float, default=0.1,
                    help="batched --congested: fraction of the streams each hot link carries")
    ap.add_argument("--chunk-sweep", type=int, nargs="*", default=[],
                    help="batched --congested: also time these heavy_chunk values")
    ap.add_argument("--heavy-chunk", type=int, default=0,
                    help="batched: nonzeros per chunk of a long link row (0: cached or default)")
    ap.add_argument("--batch-only", action="store_true",
                    help="batched: one warm-up and one timed solve only (counter runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB device copy (known bytes) for counter scaling")
    args = ap.parse_args()
    if args.cpu_to_tol and args.config not in ("tiny", "medium"):
        print("--cpu-to-tol is for the tiny and medium configs (the oracle would run "
              "for hours on the larger ones)", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2509_10722_amd import instances
    from paper_2509_10722_amd.pmp import Solver

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    if args.pattern == "batched":
        return bench_batched_congested(args, log) if args.congested else bench_batched(args, log)
    if args.pattern == "adjoint":
        return bench_adjoint(args, log)
    if args.pattern == "warmstart":
        return bench_warmstart(args, log)
    if args.pattern == "congested":
        return bench_congested(args, log)
    if args.pattern == "transit":
        return bench_transit(args, log)

    if args.calibrate_copy:
        calibrate_copy(log)

    t0 = time.perf_counter()
    inst = instances.make(args.config, scale=args.scale)
    gen_s = time.perf_counter() - t0
    st = inst.stats()
    log(f"[bench] instance {args.config}: {st} (generated in {gen_s:.1f} s)")
    inst32 = inst.rounded(np.float32)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    layout = {"auto": 0, "gather": 1, "binned": 2}[args.layout]
    solver = Solver(inst32, dtype=torch.float32, eps_abs=0.0, max_iter=max(1, args.warmup),
                    layout=layout)
    used = solver.layout_in_use()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"[bench] setup {setup_s:.2f} s")

    solver.update_params(eps_abs=0.0, max_iter=max(1, args.warmup))
    solver.solve()
    # `repeats` timed runs of `steps` iterations each (graph replays, stop
    # rule off); every run starts on a check boundary placed so that its
    # window holds a balancing iteration (rho step and u rescale, every 50).
    # The line reports the median run.
    runs = []
    for _ in range(args.repeats):
        cur = solver.residuals()[2]
        s0 = -(-cur // 10) * 10
        while (s0 + args.steps) // 50 == s0 // 50:
            s0 += 10
        if s0 > cur:
            solver.update_params(eps_abs=0.0, max_iter=s0 - cur)
            solver.solve()
        solver.update_params(eps_abs=0.0, max_iter=args.steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = solver.solve()
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
        assert res["iterations"] == args.steps
        log(f"[bench] iterations {s0 + 1}..{s0 + args.steps} in {runs[-1] * 1e3:.3f} ms, "
            f"r {res['r_norm']:.3e} s {res['s_norm']:.3e} rho {res['rho']:.4g}")
    dt = float(np.median(runs))
    ips = args.steps / dt
    log(f"[bench] median of {len(runs)} runs of {args.steps} iterations: {dt:.4f} s, "
        f"{ips:.1f} it/s")

    kt = solver.time_kernels(args.kernel_iters)
    log(f"[bench] per-kernel ms (HIP events): {kt}")
    bm = bytes_model(inst.n, inst.m, inst.nnz)
    dom = "link" if kt["link"] >= kt["stream"] else "stream"
    achieved = bm[dom] / (kt[dom] * 1e-3) / 1e9
    kname = {"link": "link_pass", "stream": "stream_pass"}[dom]
    traffic = load_traffic(kname, used, args.config)

    out_tol = {}
    if not args.no_tol:
        solver.reset()
        solver.update_params(eps_abs=1e-4, max_iter=args.tol_max_iter)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r2 = solver.solve()
        torch.cuda.synchronize()
        tt = time.perf_counter() - t0
        out_tol = {"time_to_tol_s": round(tt, 4), "iters_to_tol": int(r2["iterations"]),
                   "tol_converged": bool(r2["converged"]), "eps_abs": 1e-4}
        log(f"[bench] time to tol: {out_tol}")
    solver.close()
    del solver
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        import oracle
        k = args.cpu_iters
        ro = oracle.run(inst32, k)
        cpu = {"value": round(k / ro["loop_seconds"], 4), "unit": "iter/s",
               "cores": ro["threads"], "kind": "oracle",
               "sample": f"{k} iterations of the FP64 literal per-terminal oracle on the same "
                         f"{args.config} instance (setup excluded, {ro['loop_seconds']:.1f} s)"}
        if args.cpu_to_tol:
            # the oracle run to the stop rule itself (about 25 s for medium on
            # 16 host threads)
            rt = oracle.run(inst32, args.tol_max_iter, eps_abs=1e-4, stop=True)
            cpu["to_tol"] = {"time_s": round(rt["loop_seconds"], 3),
                             "iterations": rt["iterations"], "converged": rt["converged"]}
        if args.cpu_single_iters > 0:
            k1 = args.cpu_single_iters
            r1 = oracle.run(inst32, k1, threads=1)
            cpu["single_thread"] = {"value": round(k1 / r1["loop_seconds"], 4), "unit": "iter/s",
                                    "sample": f"{k1} iteration{'s' if k1 != 1 else ''} on one thread "
                                              f"({r1['loop_seconds']:.1f} s)"}
        log(f"[bench] cpu baseline: {cpu}")

    line = {
        "metric": METRIC, "value": round(ips, 3), "unit": "iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 5),
        "timing": {"repeats": len(runs), "statistic": "median",
                   "runs_ms": [round(1e3 * r, 3) for r in runs],
                   "window": "each run starts on a check boundary and spans a balancing "
                             "iteration (rho step and u rescale every 50)"},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config} (m={inst.m}, n={inst.n}, nnz={inst.nnz})",
                   "m": inst.m, "n": inst.n, "nnz": inst.nnz, "scale": args.scale,
                   "route_len_mean": round(st["route_len_mean"], 4),
                   "check_every": 10, "adapt_every": 50, "alpha": 1.6, "layout": used},
        "model_gbs": round(bm["iteration"] * ips / 1e9, 2),
        "model_bytes_per_iter": bm["iteration"],
        "kernel_ms": {k2: round(v, 5) for k2, v in kt.items()},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "algorithmic_bytes": bm[dom]},
        "cpu_baseline": cpu,
        "setup_s": round(setup_s, 3),
    }
    line.update(out_tol)
    if cpu and out_tol.get("tol_converged"):
        # the oracle runs the same iteration, so it needs about the same count
        cpu["time_to_tol_s_extrapolated"] = round(out_tol["iters_to_tol"] / cpu["value"], 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
