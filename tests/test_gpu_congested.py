"""Congested links (Section V-C): rows far longer than one workgroup's LDS
stage are summed by several workgroups in chunks and finished by a second
kernel in chunk order (gather layout); the binned layout balances its link
blocks by nonzeros and merges runs of one link in its LDS sums.  In FP32 with
a finite box those long rows are summed in fixed point (exact int64 sums of
x 2^F), which makes both layouts agree and repeat bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2509_10722_amd import instances as I
from tests.gpu_util import close, host, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2509_10722_amd.pmp import PMP_LAYOUT_BINNED, PMP_LAYOUT_GATHER, Solver  # noqa: E402


@pytest.fixture(scope="module")
def congested():
    base = I.medium(scale=0.2)
    return I.congested(base, link_frac=0.001, stream_frac=0.1)


def test_congested_rows_are_long(congested):
    deg = np.diff(congested.row_ptr)
    assert (deg > 8192).sum() >= 10            # several chunks per long row


@pytest.mark.parametrize("layout", [PMP_LAYOUT_GATHER, PMP_LAYOUT_BINNED])
@pytest.mark.parametrize("dtype_name,tol", [("float64", 1e-10), ("float32", 1e-5)])
def test_congested_equal_iterations(congested, dtype_name, tol, layout):
    inst = congested if dtype_name == "float64" else congested.rounded(np.float32)
    K = 120
    s = Solver(inst, dtype=getattr(torch, dtype_name), layout=layout)
    assert s.layout_in_use() == ("binned" if layout == PMP_LAYOUT_BINNED else "gather")
    s.iterate(K)
    r, sn, _ = s.residuals()
    x, lam, _ = s.solution()
    s.close()
    o = oracle.run(inst, K)
    print(f"congested {dtype_name}: x {rel(host(x), o['x']):.2e} lam {rel(host(lam), o['lam']):.2e}")
    assert rel(host(x), o["x"]) <= tol and rel(host(lam), o["lam"]) <= tol
    bits = 64 if dtype_name == "float64" else 32
    assert close(host(x), o["x"], bits) and close(host(lam), o["lam"], bits)
    assert abs(r - o["r_norm"]) <= 1e-4 * o["r_norm"]


@pytest.mark.parametrize("layout", [PMP_LAYOUT_GATHER, PMP_LAYOUT_BINNED])
def test_congested_solve_deterministic(congested, layout):
    """FP32 long rows (the congested links, 10^4 nonzeros each) are summed in
    fixed point, exactly, so the order of the binned layout's LDS adds cannot
    show: two solves are equal bit for bit in either layout."""
    inst = congested.rounded(np.float32)
    res = []
    for _ in range(2):
        s = Solver(inst, dtype=torch.float32, layout=layout, max_iter=3000)
        r = s.solve()
        x, lam, _ = s.solution()
        res.append((r["iterations"], host(x), host(lam), r["r_norm"], r["s_norm"]))
        s.close()
    print(f"congested layout {layout}: {res[0][0]} iterations, twice", flush=True)
    assert res[0][0] == res[1][0] and res[0][3:] == res[1][3:]
    assert np.array_equal(res[0][1], res[1][1]) and np.array_equal(res[0][2], res[1][2])


def test_congested_binned_equals_gather(congested):
    """Long rows: the same integer sums in both layouts; the other rows:
    exact FP64 sums of FP32 values.  The iterates agree bit for bit."""
    inst = congested.rounded(np.float32)
    out = []
    for layout in (PMP_LAYOUT_BINNED, PMP_LAYOUT_GATHER):
        s = Solver(inst, dtype=torch.float32, layout=layout)
        s.iterate(150)
        x, lam, _ = s.solution()
        out.append((host(x), host(lam), s.residuals()))
        s.close()
    (xb, lb, rb), (xg, lg, rg) = out
    print(f"congested binned vs gather: x equal {np.mean(xb == xg):.6f}, "
          f"lambda equal {np.mean(lb == lg):.6f}", flush=True)
    assert np.array_equal(xb, xg) and np.array_equal(lb, lg) and rb == rg
