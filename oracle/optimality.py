"""Converged-run checker and closed-form optima for NUM -- test infrastructure.

These are exact statements about the optimum of

    maximize sum_j U_j(x_j)  s.t.  R x <= c,  lo <= x <= hi      (eq. (2) + box)

with U_j(x) = w_j log x, w_j x or -w_j / x (Section II's utilities and the
alpha = 2 fairness it names), independent of how PMP reaches
it.  They pin the iterative oracle (and, at convergence, the HIP solver):

  kkt_report        primal feasibility, dual feasibility, complementary
                    slackness, stationarity w_j / x_j = pi_j with the path
                    price pi = R^T lambda (Section VI-B), and the duality gap
                    D(lambda) - U(x_hat) >= 0 of the Lagrangian dual.
  single_link       water-filling on the single price of one shared link.
  paper_example     the 3-link, 4-stream network of Section III-A.
  brute_force       SciPy FP64 primal (SLSQP) and, for all-log instances, the
                    dual by L-BFGS-B on D(lambda), for very small instances.
"""
from __future__ import annotations

import math

import numpy as np

LOG, LINEAR, ALPHA2 = 0, 1, 2


def csr_matvec(inst, x):
    """(R x)_l for the 0/1 pattern."""
    x = np.asarray(x, dtype=np.float64)
    rows = np.repeat(np.arange(inst.m), np.diff(inst.row_ptr))
    return np.bincount(rows, weights=x[inst.col_idx], minlength=inst.m)


def csr_rmatvec(inst, lam):
    """(R^T lambda)_j, the path price of every stream."""
    lam = np.asarray(lam, dtype=np.float64)
    rows = np.repeat(np.arange(inst.m), np.diff(inst.row_ptr))
    return np.bincount(inst.col_idx, weights=lam[rows], minlength=inst.n)


def utility(inst, x):
    """sum_j U_j(x_j); -inf if a log or alpha = 2 stream has x_j <= 0."""
    x = np.asarray(x, dtype=np.float64)
    log = inst.utility == LOG
    lin = inst.utility == LINEAR
    a2 = inst.utility == ALPHA2
    if np.any(x[log | a2] <= 0):
        return -math.inf
    return float(np.sum(inst.w[log] * np.log(x[log])) + np.sum(inst.w[lin] * x[lin])
                 - np.sum(inst.w[a2] / x[a2]))


def inner_max(inst, pi):
    """argmax and max over lo <= x <= hi of U_j(x) - pi_j x, per stream."""
    w, lo, hi = inst.w, inst.lo, inst.hi
    log = inst.utility == LOG
    lin = inst.utility == LINEAR
    a2 = inst.utility == ALPHA2
    xs = np.empty(inst.n)
    safe = np.where(pi > 0, pi, 1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        xl = np.where(pi > 0, np.clip(w / safe, lo, hi), hi)
        xa = np.where(pi > 0, np.clip(np.sqrt(w / safe), lo, hi), hi)
    xs[log] = xl[log]
    xs[a2] = xa[a2]
    xs[lin] = np.where(w[lin] > pi[lin], hi, lo)
    val = np.empty(inst.n)
    with np.errstate(divide="ignore"):
        val[log] = w[log] * np.log(xs[log]) - pi[log] * xs[log]
        val[a2] = -w[a2] / xs[a2] - pi[a2] * xs[a2]
    val[lin] = (w[lin] - pi[lin]) * xs[lin]
    return xs, val


def dual_value(inst, lam):
    """Lagrangian dual D(lambda) = lambda^T c + sum_j max_x (U_j(x) - pi_j x)."""
    lam = np.maximum(np.asarray(lam, dtype=np.float64), 0.0)
    pi = csr_rmatvec(inst, lam)
    _, val = inner_max(inst, pi)
    return float(lam @ inst.c + val.sum())


def kkt_report(inst, x, lam):
    """Optimality measures of (x, lambda); every entry -> 0 at the optimum."""
    x = np.asarray(x, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    Rx = csr_matvec(inst, x)
    lam_p = np.maximum(lam, 0.0)
    pi = csr_rmatvec(inst, lam_p)
    rep = {}
    rep["primal_infeas"] = float(np.max(np.maximum(Rx - inst.c, 0.0) / inst.c, initial=0.0))
    rep["box_violation"] = float(max(np.max(inst.lo - x, initial=0.0),
                                     np.max(x - inst.hi, initial=0.0), 0.0))
    rep["dual_infeas"] = float(np.max(np.maximum(-lam, 0.0), initial=0.0))
    scale = max(1.0, float(np.max(np.abs(lam_p * inst.c), initial=0.0)))
    rep["comp_slack"] = float(np.max(np.abs(lam_p * (inst.c - Rx)), initial=0.0) / scale)
    log = inst.utility == LOG
    a2 = inst.utility == ALPHA2
    inner = (x > inst.lo + 1e-9 * max(1.0, inst.hi if math.isfinite(inst.hi) else 1.0)) \
        & (x < inst.hi * (1 - 1e-9))
    interior = (log | a2) & inner
    if np.any(interior):
        # marginal utility U'(x): w / x (log), w / x^2 (alpha = 2); only the
        # interior entries are used, so an infinite value at x = 0 is harmless
        with np.errstate(divide="ignore", over="ignore"):
            marg = np.where(log, inst.w / np.maximum(x, 1e-300),
                            inst.w / np.maximum(x, 1e-300) ** 2)
        rep["stationarity_log"] = float(np.max(np.abs(marg[interior] - pi[interior]) /
                                               np.maximum(marg[interior], 1e-300)))
    else:
        rep["stationarity_log"] = 0.0
    # feasible point by uniform scaling (valid for lo = 0)
    ratio = float(np.max(Rx / inst.c, initial=0.0))
    x_hat = x / max(1.0, ratio)
    x_hat = np.clip(x_hat, inst.lo, inst.hi)
    U = utility(inst, x_hat)
    D = dual_value(inst, lam_p)
    rep["primal_obj"] = U
    rep["dual_obj"] = D
    rep["gap"] = D - U
    rep["rel_gap"] = (D - U) / max(1.0, abs(U))
    return rep


def single_link(w, util, cap, lo=0.0, hi=math.inf):
    """Optimum with every stream on one link of capacity `cap`.

    The optimum has one price lam >= 0 with x_j = clip(w_j/lam, lo, hi) for
    log streams and x_j = hi (w_j > lam) / lo (w_j < lam) for linear ones.
    lam = 0 when all streams at hi fit.  Otherwise lam solves
    sum_j x_j(lam) = cap, found by bisection on the monotone capacity used;
    linear streams with w_j == lam share the leftover capacity.
    Returns (x, lam).
    """
    w = np.asarray(w, dtype=np.float64)
    util = np.asarray(util)
    log = util == LOG
    n = w.size
    if math.isfinite(hi) and n * hi <= cap:
        return np.full(n, hi), 0.0

    def used(lam, strict_linear_high):
        xs = np.empty(n)
        xs[log] = np.clip(w[log] / lam, lo, hi)
        if strict_linear_high:
            xs[~log] = np.where(w[~log] > lam, hi, lo)
        else:
            xs[~log] = np.where(w[~log] >= lam, hi, lo)
        return xs

    lo_l, hi_l = 1e-300, 1.0
    while used(hi_l, True).sum() > cap:
        hi_l *= 2.0
    lo_l = hi_l / 2.0
    while used(lo_l, True).sum() <= cap and lo_l > 1e-300:
        lo_l /= 2.0
    for _ in range(200):
        mid = 0.5 * (lo_l + hi_l)
        if used(mid, True).sum() > cap:
            lo_l = mid
        else:
            hi_l = mid
    lam = hi_l
    x = used(lam, True)
    # linear streams tied at the price take the remaining capacity
    tie = (~log) & np.isclose(w, lam, rtol=1e-12, atol=0.0)
    if np.any(tie):
        left = cap - x.sum()
        share = np.clip(left / tie.sum() + lo, lo, hi)
        x[tie] = share
    return x, lam


def single_link_alpha2(w, cap):
    """One link, all alpha = 2 utilities -w_j / x_j, no binding box: KKT gives
    w_j / x_j^2 = lam, so x_j = sqrt(w_j / lam) and sum_j x_j = cap:
    x_j = cap sqrt(w_j) / sum_k sqrt(w_k), lam = (sum_k sqrt(w_k) / cap)^2."""
    rw = np.sqrt(np.asarray(w, dtype=np.float64))
    return cap * rw / rw.sum(), (rw.sum() / cap) ** 2


def paper_example(c1, c):
    """Section III-A's network, all w = 1 log utilities, capacities
    (c1, c, c).  Link 1 carries stream 1 only; links 2 and 3 are symmetric and
    share stream 2, so they carry one price p with x2 = 1/(2p),
    x3 = x4 = 1/p and x2 + x3 = c:  p = 3/(2c)."""
    p = 1.5 / c
    x = np.array([c1, c / 3.0, 2.0 * c / 3.0, 2.0 * c / 3.0])
    lam = np.array([1.0 / c1, p, p])
    return x, lam


def brute_force(inst, x0=None):
    """SciPy FP64 optimum of a very small instance.

    Primal: SLSQP on -U(x) with R x <= c and the box (log and alpha = 2
    rates kept positive).  Dual (instances without linear streams): L-BFGS-B
    on D(lambda), lambda >= 0.  Returns dict(primal_obj, x, dual_obj, lam)."""
    from scipy.optimize import minimize

    R = np.zeros((inst.m, inst.n))
    rows = np.repeat(np.arange(inst.m), np.diff(inst.row_ptr))
    R[rows, inst.col_idx] = 1.0
    log = inst.utility == LOG
    lin = inst.utility == LINEAR
    a2 = inst.utility == ALPHA2
    hi = inst.hi if math.isfinite(inst.hi) else float(np.max(inst.c)) * 2
    lo_b = np.where(log | a2, max(inst.lo, 1e-9), inst.lo)
    if x0 is None:
        x0 = np.full(inst.n, min(hi, float(np.min(inst.c))) / (inst.n + 1))

    def f(x):
        return -(np.sum(inst.w[log] * np.log(x[log])) + np.sum(inst.w[lin] * x[lin])
                 - np.sum(inst.w[a2] / x[a2]))

    def g(x):
        gr = np.empty_like(x)
        gr[log] = -inst.w[log] / x[log]
        gr[lin] = -inst.w[lin]
        gr[a2] = -inst.w[a2] / x[a2] ** 2
        return gr

    cons = [{"type": "ineq", "fun": lambda x: inst.c - R @ x, "jac": lambda x: -R}]
    res = minimize(f, x0, jac=g, bounds=list(zip(lo_b, np.full(inst.n, hi))),
                   constraints=cons, method="SLSQP",
                   options={"ftol": 1e-15, "maxiter": 2000})
    out = {"primal_obj": -float(res.fun), "x": res.x}
    if not np.any(lin):          # D is continuously differentiable without linear streams
        def D(lam):
            return dual_value(inst, lam)

        def dD(lam):
            pi = R.T @ np.maximum(lam, 0.0)
            xs, _ = inner_max(inst, pi)
            return inst.c - R @ xs

        r2 = minimize(D, np.ones(inst.m), jac=dD, bounds=[(0.0, None)] * inst.m,
                      method="L-BFGS-B", options={"ftol": 1e-15, "gtol": 1e-12,
                                                  "maxiter": 5000})
        out["dual_obj"] = float(r2.fun)
        out["lam"] = r2.x
    return out
