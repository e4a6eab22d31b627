"""Full-size parity on the large workload (m=5e6, n=2e7, nnz~1.17e8) in the
configuration bench.py times (FP32, automatic layout = binned).

The FP64 oracle runs the same instance (FP32-rounded data) through two
balancing steps; x and the prices are compared normwise and element-wise.  Properties that hold
at any size are checked after more iterations: the link flow balance of the
link-side copies and the agreement of the binned and gather layouts.
"""
import numpy as np
import pytest

import oracle
from oracle import optimality as opt
from paper_2509_10722_amd import instances as I
from tests.gpu_util import F32_ELEM, excess, host, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2509_10722_amd.pmp import PMP_LAYOUT_GATHER, Solver  # noqa: E402


@pytest.fixture(scope="module")
def large():
    return I.large().rounded(np.float32)


def test_large_equal_iterations_vs_oracle(large):
    """K = 110 spans the balancing checks at iterations 50 and 100 (rho and
    the u rescale of eqs. (17)-(18)) and ten iterations after the second."""
    K = 110
    print(f"large: {K} iterations on the GPU (binned, FP32)", flush=True)
    s = Solver(large, dtype=torch.float32)
    assert s.layout_in_use() == "binned"
    s.iterate(K)
    r, sn, it = s.residuals()
    x, lam, slack = s.solution()
    g = (host(x), host(lam), host(slack))
    hist = s.history()
    s.close()
    print(f"large: oracle {K} iterations", flush=True)
    o = oracle.run(large, K, history=True)
    its = hist[:, 0].astype(np.int64)
    assert np.array_equal(its, [50, 100, 110])
    assert np.array_equal(hist[:, 3], o["hist_rho"][its - 1])
    ex, el = rel(g[0], o["x"]), rel(g[1], o["lam"])
    qx, ql = excess(g[0], o["x"], *F32_ELEM), excess(g[1], o["lam"], *F32_ELEM)
    print(f"large K={K}: x {ex:.2e} lambda {el:.2e}, element-wise x {qx:.3f} lambda {ql:.3f}, "
          f"rho {hist[:, 3].tolist()} (oracle {o['hist_rho'][its - 1].tolist()}), "
          f"r {r:.6e} (oracle {o['r_norm']:.6e}) s {sn:.6e} (oracle {o['s_norm']:.6e})")
    assert it == K
    assert ex <= 1e-5 and el <= 1e-5 and rel(g[2], o["slack"]) <= 1e-5
    assert qx <= 1.0 and ql <= 1.0
    assert abs(r - o["r_norm"]) <= 1e-4 * o["r_norm"]
    assert abs(sn - o["s_norm"]) <= 1e-3 * o["s_norm"]


def test_large_binned_vs_gather_and_flow_balance(large):
    K = 60
    outs = []
    for layout in (0, 0, PMP_LAYOUT_GATHER):   # binned twice: run-to-run repeatability
        s = Solver(large, dtype=torch.float32, layout=layout)
        s.iterate(K)
        x, lam, _ = s.solution()
        v = s.views()
        outs.append((host(x), host(lam), s.residuals(),
                     host(v["a"]), host(v["b"]), host(v["zs"])))
        s.close()
    (xb, lb, rb, a, b, zs), (xb2, lb2, rb2, *_), (xg, lg, rg, *_) = outs
    assert np.array_equal(xb, xb2) and np.array_equal(lb, lb2) and rb == rb2
    print(f"binned vs gather after {K}: x {rel(xb, xg):.2e} lambda {rel(lb, lg):.2e}, "
          f"equal fraction {np.mean(xb == xg):.6f}")
    # exact FP64 sums of FP32 messages: the same iterates bit for bit
    assert np.array_equal(xb, xg) and np.array_equal(lb, lg)
    # (R a)_l + d_l b_l + zs_l = 0 up to FP32 rounding of the stored a, b, zs
    Ra = opt.csr_matvec(large, a)
    d = np.diff(large.row_ptr)
    resid = np.abs(Ra + d * b + zs)
    scale = np.abs(Ra) + np.abs(d * b) + np.abs(zs) + 1e-30
    assert np.quantile(resid / scale, 0.999) < 1e-5
