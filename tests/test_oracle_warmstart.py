"""Warm starts (Section V-D) on the CPU oracle.

The oracle hands back its whole iterate (z, u, p, pbar and rho) and can
start from it.  Pin: stopping after K1 iterations and restarting from the
saved iterate gives the same run as K1 + K2 iterations straight through
(fixed rho).  Experiment: after 25% of the links lose half their capacity
on a network of the paper's scaling shape (n = m / 2, routes of 5-15 links,
m = 2e4), the warm re-solve against the cold one under the absolute rule of
Section III-F and under its relative form (eps = 1e-4 of max(||p||, ||z||)
and ||rho u||).  The relative form is where the paper's roughly fivefold
warm-start gain shows; the absolute rule gives about 1.7x, as the GPU does.
"""
import numpy as np
import pytest

import oracle
from paper_2509_10722_amd import instances as I


def test_restart_from_saved_iterate_continues_the_run():
    inst = I.tiny()
    a = oracle.run(inst, 130, adapt_every=0, keep_state=True)
    b = oracle.run(inst, 70, adapt_every=0, state=a["state"], keep_state=True)
    c = oracle.run(inst, 200, adapt_every=0, keep_state=True)
    assert np.array_equal(b["x"], c["x"]) and np.array_equal(b["lam"], c["lam"])
    assert np.array_equal(b["state"], c["state"])
    assert b["r_norm"] == c["r_norm"] and b["s_norm"] == c["s_norm"]
    # rho travels with the iterate
    d = oracle.run(inst, 100, keep_state=True)
    assert d["state"][-1] == d["rho"] != 1.0
    with pytest.raises(ValueError):
        oracle.run(I.single_link([1.0], [0], 2.0, hi=10.0), 5, state=d["state"])


def _first(r, inst, eps=1e-4):
    k = np.arange(10, r["iterations"] + 1, 10)
    hr, hs = r["hist_r"][k - 1], r["hist_s"][k - 1]
    sp = np.maximum(r["hist_pnorm"], r["hist_znorm"])[k - 1]
    sd = r["hist_unorm"][k - 1]
    tol = eps * np.sqrt(inst.nnz + inst.m)
    ab = k[(hr < tol) & (hs < tol)]
    rel = k[(hr < eps * sp) & (hs < eps * sd)]
    return (int(ab[0]) if ab.size else None), (int(rel[0]) if rel.size else None)


def test_warm_start_gain_depends_on_the_stop_rule():
    base = I.paper(scale=0.002)
    rng = np.random.default_rng(7)
    K = 4000
    full = oracle.run(base, K, history=True)
    a0, r0 = _first(full, base)
    deg = I.Instance(base.name, base.m, base.n, base.row_ptr, base.col_idx,
                     np.where(rng.random(base.m) < 0.25, base.c * 0.5, base.c), base.w,
                     base.utility, base.lo, base.hi)
    cold = _first(oracle.run(deg, K, history=True), deg)
    warm = []
    for k0, rule in ((a0, 0), (r0, 1)):
        st = oracle.run(base, k0, keep_state=True)["state"]
        warm.append(_first(oracle.run(deg, K, history=True, state=st), deg)[rule])
    print(f"absolute rule: cold {cold[0]}, warm {warm[0]} ({cold[0] / warm[0]:.2f}x); "
          f"relative rule: cold {cold[1]}, warm {warm[1]} ({cold[1] / warm[1]:.2f}x)")
    assert None not in cold and None not in warm
    assert 1.2 <= cold[0] / warm[0] <= 2.5
    assert cold[1] / warm[1] >= 3.0
