#!/usr/bin/env python3
"""Write tests/golden/adjoint_fd.json: central finite differences of the FP64
oracle for the reverse-mode workload, the reference of the GPU gradient test.

Objective J(c, w) = sum_j w_j log x_j^K after K = 500 PMP iterations from the
zero state at rho = 1 (no balancing), alpha = 1.6, on the adjoint workload
(all-log utilities, routes of 3..12 links, c ~ U[1, 100]) at scale 0.1
(m = 1e4, n = 1e5) with its data rounded to FP32.  Central differences with
h = 1e-3 for 32 sampled capacities and 32 sampled weights and along one
random direction, each repeated with 2h for an estimate of its truncation
error; each pair also records whether every prox took the same branch in
the +h and -h runs (the oracle's branch digest), since a pair that
straddles a clip or slack-projection kink is not a derivative.  The
converged prices lambda* (Section VI-B, envelope: dU*/dc = lambda*) are
summarised by their norm and by the sampled entries.

With --scale 1 --coords 0 it writes adjoint_fd_scale1.json: the direction
only, on the full workload (m = 1e5, n = 1e6).  The direction is also
differenced with h = 1e-5 and 1e-7 (see small_h below); --small-h-only adds
just those to an existing file.

Only the oracle and the seeded instance generator are called.
Usage: python tests/golden/make_adjoint_fd.py [--threads N] [--scale S --coords C]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import optimality as opt  # noqa: E402
from paper_2509_10722_amd import instances as I  # noqa: E402

K, H, SEED = 500, 1e-3, 4100


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--scale", type=float, default=0.1)
    ap.add_argument("--coords", type=int, default=32,
                    help="sampled capacities and weights each (0: the direction only, "
                         "no converged prices)")
    ap.add_argument("--out", default=None)
    ap.add_argument("--small-h-only", action="store_true",
                    help="add the h = 1e-5 directional difference to an existing file")
    args = ap.parse_args()
    SCALE, NC, NW = args.scale, args.coords, args.coords
    out_path = args.out or os.path.join(
        HERE, "adjoint_fd.json" if SCALE == 0.1 else f"adjoint_fd_scale{SCALE:g}.json")
    inst = I.adjoint(scale=SCALE).rounded(np.float32)
    rng = np.random.default_rng(SEED)
    links = np.sort(rng.choice(inst.m, NC, replace=False))
    streams = np.sort(rng.choice(inst.n, NW, replace=False))
    dc = rng.normal(size=inst.m)
    dw = rng.normal(size=inst.n)

    def J_at(c, w):
        p = I.Instance(inst.name, inst.m, inst.n, inst.row_ptr, inst.col_idx, c, w,
                       inst.utility, inst.lo, inst.hi)
        o = oracle.run(p, K, adapt_every=0, threads=args.threads, branches=True)
        return opt.utility(p, o["x"]), o["branch_digest"]

    def central(dc_, dw_):
        # central differences along (dc_, dw_) with steps h and 2h: their
        # difference / 3 estimates the h one's truncation error
        # (h^2 J'''/6 + O(h^4))
        out = []
        for step in (H, 2 * H):
            jp, dp = J_at(c0 + step * dc_, w0 + step * dw_)
            jm, dm = J_at(c0 - step * dc_, w0 - step * dw_)
            out.append(((jp - jm) / (2 * step), bool(dp != dm)))
        (f1, flip1), (f2, flip2) = out
        return f1, abs(f2 - f1) / 3.0, flip1, flip1 or flip2

    t0 = time.time()
    c0, w0 = inst.c.astype(np.float64), inst.w.astype(np.float64)

    def small_h():
        # along the direction every coordinate moves, and with h = 1e-3 some
        # prox changes branch between the +h and -h runs, so the difference
        # averages the slope over kinks; smaller steps cross fewer of them
        # (the branch digest says whether any was crossed) at an FD64
        # rounding error of about eps |J| / h
        steps = []
        for hs in (1e-5, 1e-7):
            jp, dp = J_at(c0 + hs * dc, w0 + hs * dw)
            jm, dm = J_at(c0 - hs * dc, w0 - hs * dw)
            steps.append({"h": hs, "fd": (jp - jm) / (2 * hs), "branch_flip": bool(dp != dm),
                          "rounding": 2.2e-16 * abs(jp) / hs})
            print(f"direction, h = {hs:g}: {steps[-1]}", flush=True)
        return steps

    if args.small_h_only:
        with open(out_path) as f:
            out = json.load(f)
        out["direction"].pop("small_h", None)
        out["direction"]["small_steps"] = small_h()
        with open(out_path, "w") as f:
            json.dump(out, f, indent=1)
        return
    J0, _ = J_at(c0, w0)
    rows = {"c": [], "w": []}
    zc, zw = np.zeros(inst.m), np.zeros(inst.n)
    for kind, idx in (("c", links), ("w", streams)):
        for i in idx:
            e = np.zeros(inst.m if kind == "c" else inst.n)
            e[i] = 1.0
            fd, trunc, flip, flip2 = central(e, zw) if kind == "c" else central(zc, e)
            rows[kind].append({"index": int(i), "fd": fd, "trunc": trunc, "branch_flip": flip,
                               "branch_flip_2h": flip2})
            print(f"{kind}[{i}]: fd {fd:.10g} trunc {trunc:.2e} flip {flip}/{flip2}  "
                  f"({time.time() - t0:.0f} s)", flush=True)
    fd_dir, tr_dir, flip_dir, flip2_dir = central(dc, dw)
    small = small_h()
    print(f"direction: fd {fd_dir:.10g} trunc {tr_dir:.2e} flip {flip_dir}/{flip2_dir}", flush=True)
    out = {
        "workload": f"adjoint scale {SCALE} (m={inst.m}, n={inst.n}, nnz={inst.nnz}), FP32-rounded data",
        "K": K, "rho": 1.0, "alpha": 1.6, "h": H, "seed": SEED, "J": J0,
        "links": rows["c"], "streams": rows["w"],
        "direction": {"seed": SEED, "draw": "normal(size=m) for c then normal(size=n) for w, "
                      "after the two index samples", "fd": fd_dir, "trunc": tr_dir,
                      "branch_flip": flip_dir, "branch_flip_2h": flip2_dir, "small_steps": small},
    }
    if NC > 0:
        star = oracle.run(inst, 200000, eps_abs=1e-9, stop=True, threads=args.threads)
        lam = star["lam"]
        out["lambda_star"] = {"iterations": star["iterations"], "converged": star["converged"],
                              "eps_abs": 1e-9, "norm": float(np.linalg.norm(lam)),
                              "at_links": [float(lam[i]) for i in links]}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {out_path} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
