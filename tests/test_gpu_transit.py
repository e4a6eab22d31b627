"""Section VI's transit case study on the GPU: parity with the oracle at
equal iteration counts (rates, link prices and path prices) on the
case-study-sized network and on a small one, and the stationarity
w_j / x_j = pi_j of the path prices after a tight solve."""
import numpy as np
import pytest

import oracle
from oracle import optimality as opt
from paper_2509_10722_amd import instances as I
from tests.gpu_util import close, host, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2509_10722_amd.pmp import Solver  # noqa: E402


@pytest.mark.parametrize("size", ["small", "case_study"])
def test_transit_equal_iterations(size):
    if size == "small":
        inst, _ = I.transit_case_study(stations=12, T=16, edges=30, od_pairs=6, departures=4)
    else:
        inst, _ = I.transit_case_study()
    K = 500
    print(f"transit {size}: m={inst.m} n={inst.n} nnz={inst.nnz} K={K}", flush=True)
    s = Solver(inst, dtype=torch.float64)
    s.iterate(K)
    x, lam, _ = s.solution()
    pi = host(s.path_prices())
    x, lam = host(x), host(lam)
    s.close()
    o = oracle.run(inst, K)
    pi_o = opt.csr_rmatvec(inst, o["lam"])
    print(f"  x {rel(x, o['x']):.2e} lam {rel(lam, o['lam']):.2e} pi {rel(pi, pi_o):.2e}")
    assert close(x, o["x"], 64)
    assert close(lam, o["lam"], 64)
    assert close(pi, pi_o, 64)


def test_transit_path_prices_at_optimum():
    inst, meta = I.transit_case_study(stations=30, T=48, edges=120, od_pairs=20, departures=20)
    s = Solver(inst, dtype=torch.float64, eps_abs=1e-9, max_iter=300000)
    res = s.solve()
    assert res["converged"]
    x, lam, _ = s.solution()
    x = host(x)
    pi = host(s.path_prices())
    rep = opt.kkt_report(inst, x, host(lam))
    s.close()
    print(f"transit tight solve: {res['iterations']} it, {rep}")
    inner = (x > 1e-6) & (x < inst.hi * (1 - 1e-6))
    assert inner.sum() > 0.9 * inst.n
    err = np.max(np.abs(inst.w[inner] / x[inner] - pi[inner]) / (inst.w[inner] / x[inner]))
    assert err <= 1e-5
    assert rep["primal_infeas"] <= 1e-6 and abs(rep["rel_gap"]) <= 1e-6
    # of two routes of one OD pair and departure, the one with the lower path
    # price gets the larger rate (x = w / pi with w = 1)
    for k in range(len(meta["od_pairs"])):
        j = np.flatnonzero((meta["od"] == k) & (meta["t0"] == 0))
        if len(j) == 2 and abs(pi[j[0]] - pi[j[1]]) > 1e-6 * max(pi[j]):
            assert (pi[j[0]] < pi[j[1]]) == (x[j[0]] > x[j[1]])
