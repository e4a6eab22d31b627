"""Congestion (Section V-C) on the CPU oracle: where the extra iterations
come from.

A network of the paper's scaling shape (n = m / 2, routes of 5-15 links) at
m = 2e4, and the same network with 0.1% of its links each added to the
routes of 10% of the streams (hot links of degree about 1000).  The stop
rule of Section III-F is absolute (||r||, ||s|| < eps_abs sqrt(J)); the ADMM
reference the paper points to for convergence also states a relative form
(||r|| < eps ||p or z||, ||s|| < eps ||rho u||).  The oracle's per-iteration
norms give the first check iteration meeting each form:

- absolute, eps_abs = 1e-4: the congested network needs several times the
  iterations of the uncongested one;
- relative, eps = 1e-4: it needs a few hundred more, the paper's report.
"""
import numpy as np
import pytest

import oracle
from paper_2509_10722_amd import instances as I


def _first_checks(inst, K, eps=1e-4):
    r = oracle.run(inst, K, history=True)
    k = np.arange(10, K + 1, 10)
    hr, hs = r["hist_r"][k - 1], r["hist_s"][k - 1]
    scale_p = np.maximum(r["hist_pnorm"], r["hist_znorm"])[k - 1]
    scale_d = r["hist_unorm"][k - 1]
    tol = eps * np.sqrt(inst.nnz + inst.m)
    ab = k[(hr < tol) & (hs < tol)]
    rel = k[(hr < eps * scale_p) & (hs < eps * scale_d)]
    return (int(ab[0]) if ab.size else None), (int(rel[0]) if rel.size else None)


@pytest.fixture(scope="module")
def counts():
    base = I.paper(scale=0.002)
    cong = I.congested(base)
    deg = np.diff(cong.row_ptr)
    assert deg.max() >= 900 and np.sum(deg >= 900) == 20
    return _first_checks(base, 9000), _first_checks(cong, 9000)


def test_absolute_rule_slows_under_congestion(counts):
    (a0, _), (a1, _) = counts
    print(f"absolute rule: uncongested {a0}, congested {a1} iterations")
    assert a0 is not None and a1 is not None
    assert a1 >= 3 * a0


def test_relative_rule_adds_a_few_hundred(counts):
    (_, r0), (_, r1) = counts
    print(f"relative rule: uncongested {r0}, congested {r1} iterations")
    assert r0 is not None and r1 is not None
    assert 0 <= r1 - r0 <= 500
