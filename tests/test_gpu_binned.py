"""The binned message layout (PMP_LAYOUT_BINNED) against the gather layout
and the FP64 oracle.

The binned kernels add FP32 messages into FP64 LDS sums; while a sum stays
below 2^53 ulps of its smallest addend every partial sum is exact and the
result equals the gather layout's sequential FP64 sum bit for bit, which is
the case on these instances.
"""
import numpy as np
import pytest

import oracle
from paper_2509_10722_amd import instances as I
from tests.gpu_util import close, host, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2509_10722_amd.pmp import (PMP_LAYOUT_BINNED, PMP_LAYOUT_GATHER,  # noqa: E402
                                      Solver)


def _run(inst, K, dtype, layout, **kw):
    s = Solver(inst, dtype=dtype, layout=layout, **kw)
    s.iterate(K)
    r = s.residuals()
    x, lam, slack = s.solution()
    out = (host(x), host(lam), host(slack), r)
    s.close()
    return out


# large at 0.15: 3e6 streams, a few hundred stream blocks, all resident at
# once (one dispatch round); at 0.3: 6e6 streams and more stream blocks than
# the GPU holds at once, so the stream pass runs in several descending rounds
# with temporal index loads
@pytest.mark.parametrize("name,scale", [("medium", 0.2), ("large", 0.01), ("tiny", 1.0),
                                        ("large", 0.15), ("large", 0.3)])
def test_binned_equals_gather_fp32(name, scale):
    inst = I.make(name, scale=scale).rounded(np.float32)
    K = 120
    xb, lb, sb, rb = _run(inst, K, torch.float32, PMP_LAYOUT_BINNED)
    xg, lg, sg, rg = _run(inst, K, torch.float32, PMP_LAYOUT_GATHER)
    same = float(np.mean(xb == xg))
    print(f"{name}: binned vs gather x {rel(xb, xg):.2e} lam {rel(lb, lg):.2e}, "
          f"bitwise-equal x fraction {same:.6f}")
    # every FP64 partial sum of FP32 messages is exact on these instances, so
    # the LDS add order cannot show: the iterates are equal bit for bit
    assert np.array_equal(xb, xg) and np.array_equal(lb, lg) and np.array_equal(sb, sg)
    assert abs(rb[0] - rg[0]) <= 1e-5 * rg[0] and abs(rb[1] - rg[1]) <= 1e-4 * rg[1]


def test_binned_fp32_matches_oracle():
    inst = I.medium(scale=0.2).rounded(np.float32)
    K = 150
    xb, lb, _, _ = _run(inst, K, torch.float32, PMP_LAYOUT_BINNED)
    o = oracle.run(inst, K)
    assert rel(xb, o["x"]) <= 1e-5 and rel(lb, o["lam"]) <= 1e-5


def test_binned_fp64_matches_oracle():
    inst = I.tiny()
    K = 500
    xb, lb, sb, _ = _run(inst, K, torch.float64, PMP_LAYOUT_BINNED)
    o = oracle.run(inst, K)
    assert close(xb, o["x"], 64) and close(lb, o["lam"], 64)
    assert close(sb, o["slack"], 64)


def test_binned_solve_and_state():
    inst = I.tiny()
    s = Solver(inst, dtype=torch.float64, layout=PMP_LAYOUT_BINNED)
    res = s.solve()
    o = oracle.run(inst, 100000, stop=True)
    assert res["converged"] and res["iterations"] == o["iterations"]
    x, lam, _ = s.solution()
    assert close(host(x), o["x"], 64)
    st = s.get_state()
    s.iterate(30)
    x1, _, _ = s.solution()
    s.set_state(st)
    s.iterate(30)
    x2, _, _ = s.solution()
    assert torch.equal(x1, x2)
    s.close()


def test_binned_adjoint_matches_gather_adjoint():
    inst = I.tiny(scale=0.5)
    grads = []
    for layout in (PMP_LAYOUT_BINNED, PMP_LAYOUT_GATHER):
        s = Solver(inst, dtype=torch.float64, layout=layout, adapt_every=0)
        s.iterate(17)                       # iterate, then differentiate from there
        J = s.forward_ckpt(40, 9)
        gc, gw = s.backward()
        s.iterate(5)                        # the handle continues after backward
        x, _, _ = s.solution()
        grads.append((J, host(gc), host(gw), host(x)))
        s.close()
    (Jb, gcb, gwb, xb), (Jg, gcg, gwg, xg) = grads
    assert abs(Jb - Jg) <= 1e-12 * abs(Jg)
    assert rel(gcb, gcg) <= 1e-12 and rel(gwb, gwg) <= 1e-12
    assert rel(xb, xg) <= 1e-12


def test_auto_layout_threshold():
    # FP32 from 2^21 nonzeros (with m, n >= 256): binned; below, or FP64: gather
    big = I.medium(scale=0.5).rounded(np.float32)          # about 2.5e6 nonzeros
    small = I.medium(scale=0.2).rounded(np.float32)        # about 1e6
    assert big.nnz >= 1 << 21 > small.nnz
    for inst, dtype, want in ((big, torch.float32, "binned"), (small, torch.float32, "gather"),
                              (big, torch.float64, "gather")):
        s = Solver(inst, dtype=dtype)
        assert s.layout_in_use() == want
        s.close()


def test_binned_adjoint_fp32_matches_gather_adjoint():
    # FP32 forward passes agree bitwise between the layouts; the reverse sums
    # run in FP64 in both, in a different order
    inst = I.adjoint(scale=0.05).rounded(np.float32)
    out = []
    for layout in (PMP_LAYOUT_BINNED, PMP_LAYOUT_GATHER):
        s = Solver(inst, dtype=torch.float32, layout=layout, adapt_every=0)
        s.iterate(11)
        J = s.forward_ckpt(60, 7)
        gc, gw = s.backward()
        out.append((J, host(gc), host(gw)))
        s.close()
    (Jb, gcb, gwb), (Jg, gcg, gwg) = out
    print(f"fp32 adjoint: J {abs(Jb - Jg) / abs(Jg):.1e} c {rel(gcb, gcg):.1e} w {rel(gwb, gwg):.1e}")
    assert Jb == Jg
    assert rel(gcb, gcg) <= 1e-6 and rel(gwb, gwg) <= 1e-6


def _ragged_instance(seed=3):
    """Streams with empty routes (a whole range of them), links that carry no
    stream, one route of 300 links and one link on 5000 streams: the cases
    where a binned tile or block is empty and where the 8-bit length tables
    give way to the CSR/CSC lengths."""
    rng = np.random.default_rng(seed)
    m, n = 3001, 20011
    dead_links = np.arange(100, 200)
    live = np.setdiff1d(np.arange(m), dead_links)
    routes = []
    for j in range(n):
        if 5000 <= j < 10000:
            routes.append(np.zeros(0, np.int64))
            continue
        L = 300 if j == 123 else int(rng.integers(2, 9))
        routes.append(rng.choice(live, L, replace=False))
    heavy = 7
    for j in rng.choice(np.r_[0:5000, 10000:n], 5000, replace=False):
        if heavy not in routes[j]:
            routes[j] = np.append(routes[j], heavy)
    rows = np.concatenate([r for r in routes])
    cols = np.concatenate([np.full(len(r), j) for j, r in enumerate(routes)])
    order = np.lexsort((cols, rows))
    row_ptr = np.zeros(m + 1, np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    c = rng.uniform(1.0, 50.0, m)
    w = rng.uniform(0.5, 2.0, n)
    util = (rng.random(n) < 0.3).astype(np.uint8) * I.LINEAR
    return I.Instance("ragged", m, n, row_ptr, cols[order].astype(np.int32), c, w, util, 0.0, 10.0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_binned_ragged_patterns(dtype):
    npdt = np.float32 if dtype == torch.float32 else np.float64
    inst = _ragged_instance().rounded(npdt)
    deg = np.diff(inst.row_ptr)
    assert (deg == 0).sum() == 100 and deg.max() >= 5000
    K = 200
    xb, lb, sb, _ = _run(inst, K, dtype, PMP_LAYOUT_BINNED)
    xg, lg, sg, _ = _run(inst, K, dtype, PMP_LAYOUT_GATHER)
    o = oracle.run(inst, K)
    tol = 1e-5 if dtype == torch.float32 else 1e-10
    print(f"ragged {dtype}: nnz={inst.nnz} binned/oracle x {rel(xb, o['x']):.2e} "
          f"lam {rel(lb, o['lam']):.2e}; binned/gather x {rel(xb, xg):.2e}", flush=True)
    assert rel(xb, o["x"]) <= tol and rel(lb, o["lam"]) <= tol and rel(sb, o["slack"]) <= tol
    bits = 32 if dtype == torch.float32 else 64
    assert close(xb, o["x"], bits) and close(lb, o["lam"], bits)
    if dtype == torch.float32:
        # exact FP64 sums of FP32 messages in both layouts: the same iterates
        assert np.array_equal(xb, xg) and np.array_equal(lb, lg)
    # streams without links sit at the maximizer of their increasing utility
    # over the box, its upper end
    assert np.all(xb[5000:10000] == 10.0)


def test_binned_updates_and_reset_match_gather():
    """Capacity and weight updates (degradation, Section V-D) and a reset in
    the middle of a run: the binned iterates stay equal to the gathered ones
    bit for bit, including the messages rebuilt after each update."""
    inst = I.medium(scale=0.2).rounded(np.float32)
    rng = np.random.default_rng(21)
    cut = rng.random(inst.m) < 0.25
    c2 = np.where(cut, 0.5 * inst.c, inst.c).astype(np.float32)
    w2 = (inst.w * rng.uniform(0.8, 1.25, inst.n)).astype(np.float32)
    outs = []
    for layout in (PMP_LAYOUT_BINNED, PMP_LAYOUT_GATHER):
        s = Solver(inst, dtype=torch.float32, layout=layout)
        s.iterate(40)
        s.update_capacity(torch.from_numpy(c2).cuda())
        s.iterate(35)
        s.update_weights(torch.from_numpy(w2).cuda())
        s.iterate(35)
        x1, lam1, _ = s.solution()
        s.reset()
        s.iterate(20)
        x2, _, _ = s.solution()
        outs.append((host(x1), host(lam1), host(x2)))
        s.close()
    (xb, lb, xb2), (xg, lg, xg2) = outs
    assert np.array_equal(xb, xg) and np.array_equal(lb, lg) and np.array_equal(xb2, xg2)


def test_binned_mixed_utilities_with_alpha2():
    """All three utilities (log, linear, -w/x) mixed on a medium-shaped
    instance in the binned layout: the -w/x prox and the per-stream utility
    byte it reads, against the gather layout (bit for bit) and the oracle."""
    inst = I.medium(scale=0.1)
    rng = np.random.default_rng(23)
    inst.utility = rng.integers(0, 3, inst.n).astype(np.uint8)
    inst = inst.rounded(np.float32)
    assert (inst.utility == I.ALPHA2).any()
    K = 150
    xb, lb, _, _ = _run(inst, K, torch.float32, PMP_LAYOUT_BINNED)
    xg, lg, _, _ = _run(inst, K, torch.float32, PMP_LAYOUT_GATHER)
    o = oracle.run(inst, K)
    print(f"mixed utilities: binned/oracle x {rel(xb, o['x']):.2e} lam {rel(lb, o['lam']):.2e}",
          flush=True)
    assert np.array_equal(xb, xg) and np.array_equal(lb, lg)
    assert rel(xb, o["x"]) <= 1e-5 and rel(lb, o["lam"]) <= 1e-5


def test_binned_host_built_tables_for_many_stream_blocks():
    """More than 8192 stream blocks (8.5e7 streams): the tile tables are
    built on the host instead of the device; the iterates still equal the
    gather layout's bit for bit."""
    rng = np.random.default_rng(29)
    m, n = 1024, 85_000_000
    link = rng.integers(0, m, n).astype(np.int32)          # one link per stream
    order = np.argsort(link, kind="stable").astype(np.int32)
    row_ptr = np.zeros(m + 1, np.int32)
    row_ptr[1:] = np.cumsum(np.bincount(link, minlength=m))
    c = rng.uniform(1e3, 1e4, m)
    w = rng.uniform(0.5, 2.0, n)
    util = np.zeros(n, np.uint8)
    inst = I.Instance("many_stream_blocks", m, n, row_ptr, order, c, w, util, 0.0, 1e4)
    inst = inst.rounded(np.float32)
    print(f"many stream blocks: m={m} n={n} nnz={inst.nnz}", flush=True)
    outs = []
    for layout in (PMP_LAYOUT_BINNED, PMP_LAYOUT_GATHER):
        s = Solver(inst, dtype=torch.float32, layout=layout)
        s.iterate(12)
        x, lam, _ = s.solution()
        outs.append((host(x), host(lam)))
        s.close()
        del s
        torch.cuda.empty_cache()
    (xb, lb), (xg, lg) = outs
    assert np.array_equal(xb, xg) and np.array_equal(lb, lg)
