"""Control paths of the HIP library through the C ABI: the residual history
(Section III-F norms and the eqs. (17)-(18) rho schedule) against the FP64
oracle's per-iteration record, the iteration count after a reverse-mode
forward pass, rejected capacity / weight updates, and a non-finite iterate
reported as PMP_ERR_NUMERIC by the host-read status.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2509_10722_amd import instances as I
from tests.gpu_util import host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2509_10722_amd.pmp import PMP_ERR_INVALID, PMP_ERR_NUMERIC, PMPError, Solver  # noqa: E402

EPS32 = 2.0 ** -24


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_history_matches_oracle(dtype_name):
    """Every recorded check (iteration, ||r||, ||s||, rho) against the oracle's
    record of the same iteration, through a solve with balancing every 50.

    FP64: 1e-10 relative, plus an absolute floor for the cancellation in the
    link averages (y_l + ps_l -> 0 near the optimum; each link's term carries
    rounding of order eps64 |y_l|).  FP32: 1e-5 relative, plus a floor of
    8 eps32 ||p|| (the FP32 rates and slack values are rounded to eps32 of
    their size, and r, s are differences of them); rho is compared exactly."""
    dtype = getattr(torch, dtype_name)
    inst = I.tiny() if dtype_name == "float64" else I.tiny().rounded(np.float32)
    _say(f"history {dtype_name}: tiny solve, adapt 50")
    s = Solver(inst, dtype=dtype)
    res = s.solve()
    hist = s.history()
    s.close()
    K = res["iterations"]
    o = oracle.run(inst, K, history=True)
    assert res["converged"] and len(hist) == K // 10
    its = hist[:, 0].astype(np.int64)
    assert np.array_equal(its, np.arange(10, K + 1, 10))
    r_o, s_o, rho_o = (o[k][its - 1] for k in ("hist_r", "hist_s", "hist_rho"))
    if dtype_name == "float64":
        floor = 1e-12
        tol_r = 1e-10 * r_o + floor
        tol_s = 1e-10 * s_o + floor
        assert np.array_equal(hist[:, 3], rho_o)
    else:
        pn = o["hist_pnorm"][its - 1]
        tol_r = 1e-5 * r_o + 8 * EPS32 * pn
        tol_s = 1e-5 * s_o + 8 * EPS32 * rho_o * pn
        assert np.array_equal(hist[:, 3], rho_o)
    dr, ds = np.abs(hist[:, 1] - r_o), np.abs(hist[:, 2] - s_o)
    _say(f"history {dtype_name}: {len(hist)} checks, max |dr| / tol {np.max(dr / tol_r):.3f}, "
         f"max |ds| / tol {np.max(ds / tol_s):.3f}, rho changes "
         f"{int(np.sum(np.diff(hist[:, 3]) != 0))}")
    assert np.all(dr <= tol_r) and np.all(ds <= tol_s)
    assert np.sum(np.diff(hist[:, 3]) != 0) >= 2


@pytest.mark.parametrize("layout", [1, 2])
def test_solve_after_forward_ckpt_counts_iterations(layout):
    """K reverse-mode forward iterations count as iterations: a solve that
    follows reports the same iteration count, residuals and solution as a
    fresh handle started from the same state."""
    inst = I.adjoint(scale=0.02).rounded(np.float32)
    K, sk = 500, 25
    _say(f"forward_ckpt({K}, {sk}) then solve, layout {layout}")
    a = Solver(inst, dtype=torch.float32, layout=layout, adapt_every=0)
    a.forward_ckpt(K, sk)
    assert a.residuals()[2] == K
    st = a.get_state()
    ra = a.solve()
    xa, la, _ = a.solution()
    ita = a.residuals()[2]
    b = Solver(inst, dtype=torch.float32, layout=layout, adapt_every=0)
    b.set_state(st)
    rb = b.solve()
    xb, lb, _ = b.solution()
    itb = b.residuals()[2]
    a.close(); b.close()
    _say(f"  after forward_ckpt: {ra['iterations']} it; fresh from the state: {rb['iterations']} it")
    assert ra["iterations"] == rb["iterations"] and ra["iterations"] > 0
    assert ita == itb == K + ra["iterations"]
    assert ra["r_norm"] == rb["r_norm"] and ra["s_norm"] == rb["s_norm"]
    assert torch.equal(xa, xb) and torch.equal(la, lb)


@pytest.mark.parametrize("layout", [1, 2])
def test_rejected_updates_leave_instance_unchanged(layout):
    """A capacity or weight update with a zero, negative or non-finite entry
    is refused before any of it is applied; later valid updates succeed, and
    the utility types (kept in the sign of the stored weight) survive."""
    inst = I.tiny().rounded(np.float32)
    rng = np.random.default_rng(3)
    c2 = (inst.c * rng.uniform(0.5, 1.0, inst.m)).astype(np.float32)
    w2 = (inst.w * rng.uniform(0.8, 1.2, inst.n)).astype(np.float32)
    log_j = int(np.flatnonzero(inst.utility == 0)[0])
    lin_j = int(np.flatnonzero(inst.utility == 1)[0])

    def run(bad):
        s = Solver(inst, dtype=torch.float32, layout=layout)
        s.iterate(40)
        if bad:
            for arr, fn, idx, val in [(c2, s.update_capacity, 5, np.nan),
                                      (c2, s.update_capacity, 7, 0.0),
                                      (w2, s.update_weights, log_j, -1.0),
                                      (w2, s.update_weights, lin_j, np.inf)]:
                badv = arr.copy()
                badv[idx] = val
                with pytest.raises(PMPError) as e:
                    fn(badv)
                assert e.value.status == PMP_ERR_INVALID
        s.update_capacity(c2)
        s.update_weights(w2)
        s.iterate(60)
        x, lam, _ = s.solution()
        out = host(x), host(lam), s.residuals()
        s.close()
        return out

    _say(f"rejected updates, layout {layout}")
    good, after_bad = run(False), run(True)
    assert np.array_equal(good[0], after_bad[0]) and np.array_equal(good[1], after_bad[1])
    assert good[2] == after_bad[2]


@pytest.mark.parametrize("dtype_name,layout", [("float64", 1), ("float32", 1), ("float32", 2)])
def test_nonfinite_iterate_reports_numeric(dtype_name, layout):
    """An infinite rate loaded through pmp_set_state (unbounded box) reaches
    the residuals at the next check: pmp_solve and pmp_residuals return
    PMP_ERR_NUMERIC; the GPU keeps running normally."""
    dtype = getattr(torch, dtype_name)
    base = I.tiny()
    inst = I.Instance("tiny-unbounded", base.m, base.n, base.row_ptr, base.col_idx, base.c,
                      base.w, np.zeros(base.n, np.uint8), 0.0, math.inf)
    if dtype_name == "float32":
        inst = inst.rounded(np.float32)
    _say(f"non-finite iterate, {dtype_name}, layout {layout}")
    s = Solver(inst, dtype=dtype, layout=layout)
    s.iterate(20)
    st = s.get_state()
    esz = 4 if dtype_name == "float32" else 8
    a0 = np.array([np.inf], dtype=np.float32 if esz == 4 else np.float64).view(np.uint8)
    st[:esz] = torch.from_numpy(a0.copy()).to(st.device)     # a[0] = +inf
    s.set_state(st)
    with pytest.raises(PMPError) as e:
        s.solve()
    assert e.value.status == PMP_ERR_NUMERIC
    s.set_state(st)
    s.iterate(10)
    with pytest.raises(PMPError) as e:
        s.residuals()
    assert e.value.status == PMP_ERR_NUMERIC
    # a finite state afterwards solves normally
    s.reset()
    assert s.solve()["converged"]
    s.close()


def _first_check(o, eps_abs, eps_rel, J, ce=10):
    """The first check iteration at which the oracle's own norms meet
    ||r|| < eps_abs sqrt(J) + eps_rel max(||p||, ||z||) and
    ||s|| < eps_abs sqrt(J) + eps_rel ||rho u||."""
    k = np.arange(ce, len(o["hist_r"]) + 1, ce)
    tr = eps_abs * np.sqrt(J) + eps_rel * np.maximum(o["hist_pnorm"], o["hist_znorm"])[k - 1]
    ts = eps_abs * np.sqrt(J) + eps_rel * o["hist_unorm"][k - 1]
    hit = k[(o["hist_r"][k - 1] < tr) & (o["hist_s"][k - 1] < ts)]
    return int(hit[0]) if hit.size else None


@pytest.mark.parametrize("dtype_name,eps_abs,layout", [
    ("float64", 0.0, 1), ("float64", 1e-4, 1), ("float64", 0.0, 2), ("float32", 0.0, 1),
    ("float32", 0.0, 2)])
def test_relative_stop_rule_matches_oracle(dtype_name, eps_abs, layout):
    """eps_rel = 1e-4 (the relative form of the ADMM stopping rule that
    Section III-F builds on): the GPU stops at the check where the oracle's
    per-iteration norms of p, z and rho u (pinned against a per-terminal
    restatement) first meet the rule; FP64 exactly, FP32 within two checks."""
    dtype = getattr(torch, dtype_name)
    inst = I.tiny() if dtype_name == "float64" else I.tiny().rounded(np.float32)
    _say(f"relative stop rule, {dtype_name}, eps_abs {eps_abs}, layout {layout}")
    s = Solver(inst, dtype=dtype, eps_abs=eps_abs, eps_rel=1e-4, layout=layout)
    res = s.solve()
    x, _, _ = s.solution()
    s.close()
    o = oracle.run(inst, res["iterations"] + 300, history=True)
    k = _first_check(o, eps_abs, 1e-4, inst.nnz + inst.m)
    _say(f"  GPU stops at {res['iterations']}, oracle's first check meeting the rule {k}")
    assert res["converged"] and k is not None
    if dtype_name == "float64":
        assert res["iterations"] == k
    else:
        assert abs(res["iterations"] - k) <= 20
