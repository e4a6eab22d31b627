"""Congested links (Section V-C): rows far longer than one workgroup's LDS
stage are summed by several workgroups in chunks and finished by a second
kernel in chunk order (gather layout); the binned layout balances its link
blocks by nonzeros and merges runs of one link in its LDS sums."""
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


def test_congested_solve_deterministic(congested):
    # gather layout: fixed-order sums (the binned layout's LDS adds of a
    # congested link's 10^4 messages need not be exact, so their order may
    # show in the last bits)
    res = []
    for _ in range(2):
        s = Solver(congested, dtype=torch.float32, layout=PMP_LAYOUT_GATHER)
        r = s.solve()
        x, lam, _ = s.solution()
        res.append((r["iterations"], host(x), host(lam)))
        s.close()
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1]) and np.array_equal(res[0][2], res[1][2])
