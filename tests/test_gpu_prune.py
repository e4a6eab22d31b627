"""Link failure and pruning on the device (Section V-D), and path prices
(Section VI-B), through the C ABI.

The pruned pattern, maps and vectors are integer / copied data and must equal
the oracle's plain definition bit for bit.  The warm-started re-solve of the
pruned instance is compared with the oracle's solve of the oracle-pruned
instance at a tight tolerance.  Path prices after K iterations are compared
with R^T lambda of the oracle's iterate at equal K.
"""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import optimality as opt
from oracle import prune as orc_prune
from paper_2509_10722_amd import instances as I
from tests.gpu_util import close, host, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2509_10722_amd.pmp import (PMP_LAYOUT_BINNED, PMP_LAYOUT_GATHER,  # noqa: E402
                                      Solver)


def _failed(m, frac, seed):
    rng = np.random.default_rng(seed)
    return (rng.random(m) < frac).astype(np.uint8)


def _state_parts(buf, n, m, dtype):
    raw = host_bytes(buf)
    sz = 4 if dtype == torch.float32 else 8
    npdt = np.float32 if sz == 4 else np.float64
    vec = raw[:(n + 3 * m) * sz].view(npdt).astype(np.float64)
    tail = raw[(n + 3 * m) * sz:(n + 3 * m) * sz + 16]
    rho = tail[:8].view(np.float64)[0]
    it = tail[8:16].view(np.int64)[0]
    return vec[:n], vec[n:n + m], vec[n + m:n + 2 * m], vec[n + 2 * m:], rho, it


def host_bytes(t):
    return t.detach().cpu().numpy().view(np.uint8).copy()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("layout", [PMP_LAYOUT_GATHER, PMP_LAYOUT_BINNED])
def test_prune_matches_definition(dtype, layout):
    base = I.medium(scale=0.02)
    inst = I.congested(base, link_frac=0.01, stream_frac=0.5)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    inst = inst.rounded(npdt)
    s = Solver(inst, dtype=dtype, layout=layout)
    s.iterate(37)
    a, b, zs, u, rho, _ = _state_parts(s.get_state(), s.n, s.m, dtype)
    failed = _failed(inst.m, 0.05, 11)
    print(f"prune: m={inst.m} n={inst.n} nnz={inst.nnz} failed={int(failed.sum())} "
          f"layout={layout} dtype={dtype}", flush=True)
    p, lmap, smap = s.prune(failed)
    ref = orc_prune.prune(inst, failed)
    pi = p.instance
    assert (pi.m, pi.n, pi.nnz) == (ref["m"], ref["n"], ref["nnz"])
    assert np.array_equal(pi.row_ptr.cpu().numpy(), ref["row_ptr"])
    assert np.array_equal(pi.col_idx.cpu().numpy(), ref["col_idx"])
    assert np.array_equal(lmap.cpu().numpy(), ref["link_map"])
    assert np.array_equal(smap.cpu().numpy(), ref["stream_map"])
    assert np.array_equal(host(pi.c), ref["c"].astype(np.float64))
    assert np.array_equal(host(pi.w), ref["w"].astype(np.float64))
    assert np.array_equal(pi.utility.cpu().numpy(), ref["utility"])
    # warm start: the iterate restricted to the survivors, rho carried
    a2, b2, zs2, u2, rho2, it2 = _state_parts(p.get_state(), p.n, p.m, dtype)
    ra, rb, rz, ru = orc_prune.restrict_state(a, b, zs, u, ref["link_map"], ref["stream_map"])
    assert np.array_equal(a2, ra) and np.array_equal(b2, rb)
    assert np.array_equal(zs2, rz) and np.array_equal(u2, ru)
    assert rho2 == rho and it2 == 0
    p.close()
    s.close()


def test_prune_warm_resolve_matches_oracle():
    # all-log utilities: the optimal rates are unique
    inst = I.adjoint(scale=0.002)
    s = Solver(inst, dtype=torch.float64, eps_abs=1e-9, max_iter=200000)
    r0 = s.solve()
    assert r0["converged"]
    failed = _failed(inst.m, 0.1, 5)
    p, lmap, smap = s.prune(failed)
    r1 = p.solve()
    assert r1["converged"]
    x, lam, _ = p.solution()
    ref = orc_prune.prune(inst, failed)
    pinst = I.Instance("pruned", ref["m"], ref["n"], ref["row_ptr"], ref["col_idx"],
                       ref["c"], ref["w"], ref["utility"], inst.lo, inst.hi)
    o = oracle.run(pinst, 400000, eps_abs=1e-9, stop=True)
    assert o["converged"]
    print(f"warm re-solve: {r1['iterations']} it (oracle cold {o['iterations']}); "
          f"x {rel(host(x), o['x']):.2e}", flush=True)
    assert rel(host(x), o["x"]) <= 1e-5
    rep = opt.kkt_report(pinst, host(x), host(lam))
    assert rep["primal_infeas"] <= 1e-6 and rep["rel_gap"] <= 1e-6
    p.close()
    s.close()


def test_prune_edge_cases():
    inst = I.tiny(seed=2)
    s = Solver(inst, dtype=torch.float64)
    s.iterate(10)
    # nothing fails: the same instance, identity maps, same iterate
    p, lmap, smap = s.prune(np.zeros(inst.m, np.uint8))
    assert (p.m, p.n, p.nnz) == (inst.m, inst.n, inst.nnz)
    assert np.array_equal(lmap.cpu().numpy(), np.arange(inst.m))
    assert np.array_equal(smap.cpu().numpy(), np.arange(inst.n))
    p.close()
    # every link fails: zero sizes reported (a problem with m = 0 cannot be set up)
    lib = s.lib
    nb = ctypes.c_size_t()
    assert lib.pmp_prune_workspace_size(s.handle, ctypes.byref(nb)) == 0
    dev = dict(device="cuda")
    ws = torch.empty(nb.value, dtype=torch.uint8, **dev)
    f = torch.ones(inst.m, dtype=torch.uint8, **dev)
    rp = torch.full((inst.m + 1,), -7, dtype=torch.int32, **dev)
    ci = torch.empty(inst.nnz, dtype=torch.int32, **dev)
    c = torch.empty(inst.m, dtype=torch.float64, **dev)
    w = torch.empty(inst.n, dtype=torch.float64, **dev)
    ut = torch.empty(inst.n, dtype=torch.uint8, **dev)
    lm = torch.empty(inst.m, dtype=torch.int32, **dev)
    sm = torch.empty(inst.n, dtype=torch.int32, **dev)
    st = torch.empty(s.state_size(), dtype=torch.uint8, **dev)
    sizes = (ctypes.c_int64 * 3)()
    args = [s.handle, f.data_ptr(), ws.data_ptr(), nb.value, rp.data_ptr(), ci.data_ptr(),
            c.data_ptr(), w.data_ptr(), ut.data_ptr(), lm.data_ptr(), sm.data_ptr(),
            st.data_ptr(), sizes]
    assert lib.pmp_prune(*args) == 0
    assert list(sizes) == [0, 0, 0]
    assert int(rp[0]) == 0
    # a short workspace is refused before any work is queued
    args[3] = nb.value - 1
    assert lib.pmp_prune(*args) != 0
    s.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_path_prices_equal_iterations(dtype):
    npdt = np.float32 if dtype == torch.float32 else np.float64
    inst = I.tiny(seed=1).rounded(npdt)
    K = 300
    s = Solver(inst, dtype=dtype)
    s.iterate(K)
    pi = host(s.path_prices())
    s.close()
    o = oracle.run(inst, K)
    ref = opt.csr_rmatvec(inst, o["lam"])
    err = rel(pi, ref)
    print(f"path prices {dtype}: {err:.2e}", flush=True)
    assert err <= (1e-10 if dtype == torch.float64 else 1e-5)
    assert close(pi, ref, 64 if dtype == torch.float64 else 32)


def test_path_prices_equal_marginal_utility_at_optimum():
    # KKT stationarity (Section VI-B): w_j / x_j = pi_j for interior log rates
    inst = I.tiny(seed=0)
    s = Solver(inst, dtype=torch.float64, eps_abs=1e-10, max_iter=200000)
    assert s.solve()["converged"]
    x, _, _ = s.solution()
    x = host(x)
    pi = host(s.path_prices())
    s.close()
    inner = (inst.utility == I.LOG) & (x > 1e-6) & (x < inst.hi * (1 - 1e-6))
    assert inner.sum() > 10
    err = np.max(np.abs(inst.w[inner] / x[inner] - pi[inner]) / (inst.w[inner] / x[inner]))
    assert err <= 1e-5
