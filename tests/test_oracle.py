"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test names the passage it follows.  None re-types the oracle's own
formulas: they compare with 1-D numerical minimisation, closed-form optima,
KKT conditions, duality, brute force, and structural invariants.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import oracle
from oracle import optimality as opt
from paper_2509_10722_amd import instances as I


# ---- P1: each prox closed form (Section III-E) vs 1-D minimisation ---------

def _numeric_prox(f, zetas, rho, lo, hi):
    obj = lambda x: f(x) + 0.5 * rho * np.sum((x - zetas) ** 2)
    res = minimize_scalar(obj, bounds=(lo, hi), method="bounded",
                          options={"xatol": 1e-13, "maxiter": 5000})
    # the bounded method never evaluates the endpoints; compare with them
    cands = [(res.fun, res.x), (obj(lo), lo), (obj(hi), hi)]
    return min(cands)[1]


@pytest.mark.parametrize("seed", range(40))
def test_prox_log_matches_minimisation(seed):
    rng = np.random.default_rng(seed)
    L = int(rng.integers(1, 12))
    zetas = rng.normal(0, 3, L) * rng.choice([0.01, 1, 30])
    w = rng.uniform(0.1, 3)
    rho = rng.choice([0.1, 1.0, 7.0])
    lo, hi = 1e-12, float(rng.choice([5.0, 50.0, 1e3]))
    x = oracle.prox_log(float(zetas.sum()), L, w, rho, 0.0, hi)
    xr = _numeric_prox(lambda v: -w * math.log(v), zetas, rho, lo, hi)
    assert abs(x - xr) <= 1e-6 * max(1.0, abs(xr))


@pytest.mark.parametrize("seed", range(40))
def test_prox_linear_matches_minimisation(seed):
    rng = np.random.default_rng(100 + seed)
    L = int(rng.integers(1, 12))
    zetas = rng.normal(0, 3, L)
    w = rng.uniform(0.1, 3)
    rho = rng.choice([0.1, 1.0, 7.0])
    lo, hi = float(rng.choice([0.0, 0.5])), float(rng.choice([2.0, 10.0]))
    x = oracle.prox_linear(float(zetas.sum()), L, w, rho, lo, hi)
    xr = _numeric_prox(lambda v: -w * v, zetas, rho, lo, hi)
    assert abs(x - xr) <= 1e-6 * max(1.0, abs(xr))


def test_prox_slack_is_projection():
    # indicator of p + c >= 0: the prox is the projection onto [-c, inf)
    for zeta, c in [(-5.0, 2.0), (-2.0, 2.0), (0.3, 2.0), (-1.9, 2.0)]:
        xr = _numeric_prox(lambda v: 0.0, np.array([zeta]), 1.0, -c, 10.0)
        assert abs(oracle.prox_slack(zeta, c) - xr) < 1e-7


def test_prox_log_no_cancellation_for_very_negative_argument():
    # S << 0: the minimiser is ~ w / (rho |S|); check against the root of the
    # stationarity condition rho L x^2 - rho S x - w = 0 found by bisection
    S, L, w, rho = -1e7, 3, 1.5, 2.0
    x = oracle.prox_log(S, L, w, rho, 0.0, math.inf)
    g = lambda v: rho * L * v * v - rho * S * v - w
    a, b = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (a + b)
        a, b = (mid, b) if g(mid) < 0 else (a, mid)
    assert abs(x - a) <= 1e-12 * a


def test_empty_route_takes_upper_bound():
    assert oracle.prox_log(0.0, 0, 1.0, 1.0, 0.0, 7.0) == 7.0
    assert oracle.prox_linear(0.0, 0, 1.0, 1.0, 0.0, 7.0) == 7.0


# ---- P2: one link, all log: x_j = w_j c / sum w, lambda = sum w / c --------

def test_single_link_all_log_closed_form():
    w = np.array([0.5, 1.0, 1.7, 2.0, 0.9])
    cap = 6.0
    inst = I.single_link(w, [0] * 5, cap)
    r = oracle.run(inst, 20000, eps_abs=1e-12, stop=True, check_every=10)
    assert r["converged"]
    np.testing.assert_allclose(r["x"], w * cap / w.sum(), rtol=1e-8)
    np.testing.assert_allclose(r["lam"], [w.sum() / cap], rtol=1e-8)
    np.testing.assert_allclose(r["slack"], [0.0], atol=1e-8)


# ---- P3: one link, mixed log/linear with a box: water-filling -------------

@pytest.mark.parametrize("seed", range(6))
def test_single_link_mixed_waterfilling(seed):
    rng = np.random.default_rng(seed)
    n = 8
    util = rng.integers(0, 2, n)
    w = rng.uniform(0.3, 2.0, n)
    cap, hi = float(rng.uniform(2, 12)), 3.0
    inst = I.single_link(w, util, cap, 0.0, hi)
    r = oracle.run(inst, 60000, eps_abs=1e-11, stop=True, check_every=10)
    assert r["converged"]
    xs, lam = opt.single_link(w, util, cap, 0.0, hi)
    assert abs(opt.utility(inst, r["x"]) - opt.utility(inst, xs)) < 1e-7
    log = util == 0
    np.testing.assert_allclose(r["x"][log], xs[log], rtol=1e-6, atol=1e-8)
    assert abs(r["lam"][0] - lam) < 1e-6 * max(1.0, lam)


# ---- P4: the paper's 3-link, 4-stream example (Section III-A) -------------

@pytest.mark.parametrize("c1,c", [(1.0, 3.0), (2.5, 1.2), (0.7, 9.0)])
def test_paper_example(c1, c):
    inst = I.paper_example(c1, c)
    r = oracle.run(inst, 20000, eps_abs=1e-12, stop=True, check_every=10)
    assert r["converged"]
    x, lam = opt.paper_example(c1, c)
    np.testing.assert_allclose(r["x"], x, rtol=1e-8)
    np.testing.assert_allclose(r["lam"], lam, rtol=1e-7)


def test_paper_example_golden():
    """Fixture tests/golden/paper_example.txt (derived by hand, see file)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_example.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    vals = {r[0]: np.array([float(v) for v in r[1:]]) for r in rows}
    inst = I.paper_example(vals["c"][0], vals["c"][1])
    r = oracle.run(inst, 20000, eps_abs=1e-12, stop=True, check_every=10)
    np.testing.assert_allclose(r["x"], vals["x"], rtol=1e-8)
    np.testing.assert_allclose(r["lam"], vals["lambda"], rtol=1e-7)


# ---- P5: disjoint blocks decouple (fixed rho) ------------------------------

def test_block_structure_decouples():
    a = I.paper_example(1.0, 3.0)
    b = I.tiny(scale=0.1)
    b.lo, b.hi = a.lo, a.hi = 0.0, 10.0
    u = I.block_diagonal([a, b])
    kw = dict(adapt_every=0, alpha=1.6)
    ru, ra, rb = oracle.run(u, 300, **kw), oracle.run(a, 300, **kw), oracle.run(b, 300, **kw)
    np.testing.assert_array_equal(ru["x"], np.concatenate([ra["x"], rb["x"]]))
    np.testing.assert_array_equal(ru["lam"], np.concatenate([ra["lam"], rb["lam"]]))


# ---- P6/P7: KKT and duality gap at convergence (Section VI-B) -------------

def test_tiny_converges_to_kkt_point():
    inst = I.tiny()
    r = oracle.run(inst, 100000, eps_abs=1e-9, stop=True, check_every=10)
    assert r["converged"]
    rep = opt.kkt_report(inst, r["x"], r["lam"])
    assert rep["primal_infeas"] < 1e-6
    assert rep["dual_infeas"] < 1e-6
    assert rep["comp_slack"] < 1e-6
    assert rep["stationarity_log"] < 1e-5
    assert -1e-9 <= rep["gap"] and rep["rel_gap"] < 1e-6


def test_tiny_stops_below_tolerance_and_records_history():
    inst = I.tiny()
    r = oracle.run(inst, 5000, stop=True, history=True)
    assert r["converged"]
    k = r["iterations"]
    assert k % 10 == 0
    assert r["hist_r"][-1] < r["eps_tol"] and r["hist_s"][-1] < r["eps_tol"]
    J = inst.nnz + inst.m
    assert abs(r["eps_tol"] - 1e-4 * math.sqrt(J)) < 1e-15
    # no earlier check iteration met the rule
    for i in range(9, k - 1, 10):
        assert not (r["hist_r"][i] < r["eps_tol"] and r["hist_s"][i] < r["eps_tol"])


def test_rho_balancing_schedule():
    """Eq. (6): rho changes only every 50 iterations, by gamma or 1/gamma,
    in the direction that balances ||r|| and ||s|| (mu = 2)."""
    inst = I.tiny()
    r = oracle.run(inst, 1000, history=True, adapt_every=50)
    rho, hr, hs = r["hist_rho"], r["hist_r"], r["hist_s"]
    changed = 0
    for k in range(1, len(rho)):
        if rho[k] != rho[k - 1]:
            assert k % 50 == 0
            ratio = rho[k] / rho[k - 1]
            i = k - 1                      # decision taken at iteration k
            if hr[i] > 2 * hs[i]:
                assert abs(ratio - 1.1) < 1e-12
            else:
                assert hs[i] > 2 * hr[i] and abs(ratio - 1 / 1.1) < 1e-12
            changed += 1
        elif k % 50 == 0:
            i = k - 1
            assert not (hr[i] > 2 * hs[i]) and not (hs[i] > 2 * hr[i])
    assert changed > 0


def test_prices_invariant_under_rescale():
    """u is the scaled dual y / rho: a rho schedule changes u but, at
    convergence, the link prices rho u must be the same optimum."""
    inst = I.tiny()
    a = oracle.run(inst, 100000, eps_abs=1e-9, stop=True, adapt_every=50)
    b = oracle.run(inst, 100000, eps_abs=1e-9, stop=True, adapt_every=0)
    assert a["converged"] and b["converged"]
    np.testing.assert_allclose(a["lam"], b["lam"], atol=1e-5)


# ---- P8: brute force on very small instances -------------------------------

def _tiny_random(seed, n=6, m=4, all_log=False):
    rng = np.random.default_rng(seed)
    pairs = set()
    link, stream = [], []
    for j in range(n):
        L = int(rng.integers(1, m + 1))
        for l in rng.choice(m, L, replace=False):
            link.append(int(l)); stream.append(j)
    row_ptr, col_idx = I.csr_from_pairs(m, n, np.array(link), np.array(stream))
    util = np.zeros(n, np.uint8) if all_log else rng.integers(0, 2, n).astype(np.uint8)
    w = rng.uniform(0.5, 2.0, n)
    return I.Instance("bf", m, n, row_ptr, col_idx, rng.uniform(1, 5, m), w, util, 0.0, 4.0)


@pytest.mark.parametrize("seed", range(8))
def test_brute_force_objective(seed):
    inst = _tiny_random(seed, all_log=(seed % 2 == 0))
    r = oracle.run(inst, 200000, eps_abs=1e-10, stop=True)
    assert r["converged"]
    bf = opt.brute_force(inst)
    U = opt.utility(inst, r["x"])
    assert abs(U - bf["primal_obj"]) < 1e-6 * max(1.0, abs(U))
    if "dual_obj" in bf:
        assert abs(U - bf["dual_obj"]) < 1e-6 * max(1.0, abs(U))
    rep = opt.kkt_report(inst, r["x"], r["lam"])
    assert rep["rel_gap"] < 1e-7


# ---- P9: link flow balance 1^T z_l = 0 every iteration (Section III-C) ----

def test_zsum_invariant():
    r = oracle.run(I.tiny(), 500, alpha=1.6)
    assert r["zsum_worst"] < 1e-12


# ---- P11: fixed point ------------------------------------------------------

def test_fixed_point():
    inst = I.tiny()
    a = oracle.run(inst, 100000, eps_abs=1e-10, stop=True, adapt_every=0)
    k = a["iterations"]
    b = oracle.run(inst, k + 1, adapt_every=0)
    assert np.max(np.abs(a["x"] - b["x"])) < 1e-7
    assert np.max(np.abs(a["lam"] - b["lam"])) < 1e-7


def test_thread_count_does_not_change_results():
    inst = I.tiny()
    a = oracle.run(inst, 200, threads=1)
    b = oracle.run(inst, 200, threads=4)
    np.testing.assert_array_equal(a["x"], b["x"])
    np.testing.assert_array_equal(a["lam"], b["lam"])
    assert a["r_norm"] == b["r_norm"] and a["s_norm"] == b["s_norm"]


# ---- over-relaxed updates as printed (Section III-G) -----------------------

def _printed_updates(inst, iters, alpha, rho, adapt_every=0, mu=2.0, gamma=1.1,
                     eps_abs=None, check_every=10):
    """Per-terminal restatement of PMP exactly as the paper prints it, written
    with NumPy over a terminal list (independent of the oracle's C loops):

      p = prox(z - u)                      Section III-E closed forms
      z_l <- alpha (p_l - pbar_l) + (1 - alpha) z_l,  u_l <- u_l + alpha pbar_l
                                           over-relaxed updates, Section III-G
      r_t = pbar_l(t),  s_t = rho ((p_t - pbar_l(t)) - (p_t' - pbar_l(t)'))
                                           residuals, Section III-F (p', pbar'
                                           the previous iteration's values)
      stop when ||r||, ||s|| < eps_abs sqrt(J) at multiples of check_every
      every adapt_every iterations: rho <- gamma rho if ||r|| > mu ||s||,
      rho <- rho / gamma if ||s|| > mu ||r|| (eq. (17)), then
      u <- (rho_old / rho_new) u (eq. (18))

    u is held as one value per link (it starts at 0 and every update adds the
    same pbar_l to all of a link's terminals).  Returns x, the prices rho u
    and the per-iteration history of ||r||, ||s|| and the rho used, plus the
    textbook ADMM residuals ||p - z|| and rho ||z - z_prev|| (valid as
    residuals of the consensus form at alpha = 1) and the stop iteration."""
    m, n = inst.m, inst.n
    row_ptr = np.asarray(inst.row_ptr, np.int64)
    deg = np.diff(row_ptr)
    # traffic terminals in CSR order, then one slack terminal per link
    t_link = np.concatenate([np.repeat(np.arange(m), deg), np.arange(m)])
    t_stream = np.concatenate([np.asarray(inst.col_idx, np.int64), -np.ones(m, np.int64)])
    traffic = t_stream >= 0
    Jn = len(t_link)
    cnt = np.bincount(t_link, minlength=m).astype(float)          # |l| = d_l + 1
    L = np.bincount(t_stream[traffic], minlength=n).astype(float)  # |sigma_j|
    w = np.asarray(inst.w, float)
    util = np.asarray(inst.utility)
    z = np.zeros(Jn)
    u = np.zeros(m)
    p_prev = np.zeros(Jn)
    pbar_prev = np.zeros(m)
    x = np.zeros(n)
    hist = {"r": [], "s": [], "rho": [], "r_admm": [], "s_admm": [], "pn": [], "zn": [], "un": []}
    stop_at = None
    eps_tol = None if eps_abs is None else eps_abs * math.sqrt(Jn)
    for k in range(1, iters + 1):
        zeta = z - u[t_link]
        S = np.bincount(t_stream[traffic], weights=zeta[traffic], minlength=n)
        for j in range(n):
            if L[j] == 0:
                x[j] = inst.hi
                continue
            if util[j] == 0:
                q = math.sqrt(S[j] ** 2 + 4 * w[j] * L[j] / rho)
                xj = (S[j] + q) / (2 * L[j]) if S[j] >= 0 else 2 * w[j] / (rho * (q - S[j]))
            else:
                xj = (S[j] + w[j] / rho) / L[j]
            x[j] = min(max(xj, inst.lo), inst.hi)
        p = np.where(traffic, x[np.maximum(t_stream, 0)],
                     np.maximum(zeta, -np.asarray(inst.c, float)[t_link]))
        pbar = np.bincount(t_link, weights=p, minlength=m) / cnt
        z_prev = z
        z = alpha * (p - pbar[t_link]) + (1 - alpha) * z
        u = u + alpha * pbar
        r_vec = pbar[t_link]
        s_vec = rho * ((p - pbar[t_link]) - (p_prev - pbar_prev[t_link]))
        hist["r"].append(float(np.sqrt(np.sum(r_vec ** 2))))
        hist["s"].append(float(np.sqrt(np.sum(s_vec ** 2))))
        hist["rho"].append(rho)
        hist["r_admm"].append(float(np.linalg.norm(p - z)))
        hist["s_admm"].append(float(rho * np.linalg.norm(z - z_prev)))
        hist["pn"].append(float(np.linalg.norm(p)))
        hist["zn"].append(float(np.linalg.norm(z)))
        hist["un"].append(float(rho * np.sqrt(np.sum(cnt * u * u))))
        p_prev, pbar_prev = p, pbar
        rn, sn = hist["r"][-1], hist["s"][-1]
        if eps_tol is not None and k % check_every == 0 and rn < eps_tol and sn < eps_tol:
            stop_at = k
            break
        if adapt_every and k % adapt_every == 0:
            new = gamma * rho if rn > mu * sn else (rho / gamma if sn > mu * rn else rho)
            u = u * (rho / new)
            rho = new
    hist = {key: np.array(v) for key, v in hist.items()}
    return x, rho * u, hist, stop_at


@pytest.mark.parametrize("alpha", [1.0, 1.6, 1.9])
def test_matches_printed_overrelaxed_updates(alpha):
    for inst in (I.paper_example(1.0, 3.0), I.tiny(scale=0.05)):
        xp, lp, _, _ = _printed_updates(inst, 60, alpha, 1.3)
        r = oracle.run(inst, 60, alpha=alpha, rho0=1.3, adapt_every=0)
        np.testing.assert_allclose(r["x"], xp, rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(r["lam"], lp, rtol=1e-10, atol=1e-12)


def test_residuals_and_rho_schedule_match_restatement():
    """Section III-F residuals and the Section III-G balancing schedule
    (eqs. (17)-(18)) of the oracle against the per-terminal restatement:
    300 iterations of the tiny instance at alpha = 1.6 with balancing every
    50 iterations, which changes rho several times."""
    inst = I.tiny()
    K = 300
    r = oracle.run(inst, K, alpha=1.6, history=True, adapt_every=50)
    xp, lp, h, _ = _printed_updates(inst, K, 1.6, 1.0, adapt_every=50)
    changes = int(np.sum(h["rho"][1:] != h["rho"][:-1]))
    assert changes >= 2, changes
    np.testing.assert_array_equal(r["hist_rho"], h["rho"])
    np.testing.assert_allclose(r["hist_r"], h["r"], rtol=1e-10)
    np.testing.assert_allclose(r["hist_s"], h["s"], rtol=1e-10)
    np.testing.assert_allclose(r["hist_pnorm"], h["pn"], rtol=1e-10)
    np.testing.assert_allclose(r["hist_znorm"], h["zn"], rtol=1e-10)
    np.testing.assert_allclose(r["hist_unorm"], h["un"], rtol=1e-10)
    np.testing.assert_allclose(r["x"], xp, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(r["lam"], lp, rtol=1e-9, atol=1e-12)


def test_residuals_are_admm_residuals_at_alpha_one():
    """At alpha = 1 the consensus ADMM's own residuals are r = p - z and
    s = rho (z - z_prev) (the z-update then gives z = p - pbar); the
    oracle's Section III-F norms must equal them, through rho changes."""
    inst = I.tiny(scale=0.25)
    K = 250
    r = oracle.run(inst, K, alpha=1.0, history=True, adapt_every=50)
    _, _, h, _ = _printed_updates(inst, K, 1.0, 1.0, adapt_every=50)
    assert np.sum(h["rho"][1:] != h["rho"][:-1]) >= 1
    np.testing.assert_allclose(r["hist_r"], h["r_admm"], rtol=1e-9)
    np.testing.assert_allclose(r["hist_s"], h["s_admm"], rtol=1e-9)


@pytest.mark.parametrize("alpha,adapt", [(1.6, 50), (1.0, 0)])
def test_stop_iteration_matches_restatement(alpha, adapt):
    """The stop rule of Section III-F (both norms below 1e-4 sqrt(J) at a
    check) fires at the same iteration in the oracle and the restatement."""
    inst = I.tiny()
    r = oracle.run(inst, 5000, alpha=alpha, adapt_every=adapt, stop=True, eps_abs=1e-4)
    _, _, h, k = _printed_updates(inst, 5000, alpha, 1.0, adapt_every=adapt, eps_abs=1e-4)
    assert r["converged"] and k is not None
    assert r["iterations"] == k
    assert abs(r["rho"] - h["rho"][-1]) <= 1e-15 * r["rho"]


# ---- alpha = 2 fairness (named in Section II) -------------------------------

@pytest.mark.parametrize("seed", range(30))
def test_prox_alpha2_matches_minimisation(seed):
    rng = np.random.default_rng(500 + seed)
    L = int(rng.integers(1, 12))
    zetas = rng.normal(0, 3, L) * rng.choice([0.01, 1, 30])
    w = rng.uniform(0.1, 3)
    rho = rng.choice([0.1, 1.0, 7.0])
    hi = float(rng.choice([5.0, 50.0, 1e3]))
    x = oracle.prox_alpha2(float(zetas.sum()), L, w, rho, 0.0, hi)
    xr = _numeric_prox(lambda v: w / v, zetas, rho, 1e-9, hi)
    assert abs(x - xr) <= 1e-6 * max(1.0, abs(xr))


def test_single_link_alpha2_closed_form():
    w = np.array([0.5, 1.0, 1.7, 2.0])
    inst = I.single_link(w, [2] * 4, 6.0)
    r = oracle.run(inst, 50000, eps_abs=1e-12, stop=True)
    assert r["converged"]
    x, lam = opt.single_link_alpha2(w, 6.0)
    np.testing.assert_allclose(r["x"], x, rtol=1e-8)
    np.testing.assert_allclose(r["lam"], [lam], rtol=1e-7)


@pytest.mark.parametrize("seed", range(4))
def test_alpha2_mixed_brute_force_and_kkt(seed):
    inst = _tiny_random(30 + seed)
    rng = np.random.default_rng(seed)
    inst.utility = rng.integers(0, 3, inst.n).astype(np.uint8)
    r = oracle.run(inst, 300000, eps_abs=1e-10, stop=True)
    assert r["converged"]
    bf = opt.brute_force(inst)
    U = opt.utility(inst, r["x"])
    assert abs(U - bf["primal_obj"]) < 1e-6 * max(1.0, abs(U))
    rep = opt.kkt_report(inst, r["x"], r["lam"])
    assert rep["rel_gap"] < 1e-7 and rep["stationarity_log"] < 1e-5
