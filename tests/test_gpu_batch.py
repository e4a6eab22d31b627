"""Batched persistent solves (pmp_batch_*) against plain solves and the
oracle."""
import numpy as np
import pytest

import oracle
from paper_2509_10722_amd import instances as I
from tests.gpu_util import close, host, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2509_10722_amd.pmp import BatchSolver, Solver, batch_options_default  # noqa: E402


def _small_batch(count=6, scale=0.01, seed=3):
    return I.batched(seed=seed, count=count, scale=scale)


def test_batch_matches_plain_solves_fp64():
    insts = _small_batch()
    b = BatchSolver(insts, dtype=torch.float64)
    res = b.solve(20000)
    for k, inst in enumerate(insts):
        s = Solver(inst, dtype=torch.float64)
        r = s.solve()
        x, lam, _ = s.solution()
        xb, lb, _ = b.solution(k)
        print(f"instance {k} (m={inst.m}): batch {res[k]['iterations']} it, plain {r['iterations']} it")
        assert res[k]["converged"] and r["converged"]
        assert res[k]["iterations"] == r["iterations"]
        assert torch.equal(x, xb) and torch.equal(lam, lb)
        s.close()
    b.close()


def test_batch_fp32_equal_iterations_vs_oracle():
    insts = [i.rounded(np.float32) for i in _small_batch(count=4)]
    K = 120
    b = BatchSolver(insts, dtype=torch.float32, eps_abs=0.0)
    res = b.solve(K)
    for k, inst in enumerate(insts):
        assert res[k]["iterations"] == K and not res[k]["converged"]
        o = oracle.run(inst, K)
        x, lam, _ = b.solution(k)
        assert rel(host(x), o["x"]) <= 1e-5 and rel(host(lam), o["lam"]) <= 1e-5
    b.close()


def test_tile_caps_do_not_change_iterates():
    insts = _small_batch(count=5)
    outs = []
    for caps in ((64, 64, 64), (4096, 4096, 4096), (512, 1024, 2048)):
        b = BatchSolver(insts, dtype=torch.float64, eps_abs=0.0,
                        options=batch_options_default(tile_cap=caps))
        b.solve(90)
        outs.append([host(b.solution(k)[0]) for k in range(len(insts))])
        b.close()
    for o in outs[1:]:
        for a, c in zip(outs[0], o):
            assert np.array_equal(a, c)


def test_batch_reset_and_continue():
    insts = _small_batch(count=3)
    b = BatchSolver(insts, dtype=torch.float64, eps_abs=0.0)
    b.solve(50)
    b.solve(30)
    x1 = [host(b.solution(k)[0]) for k in range(3)]
    b.reset()
    b.solve(80)
    x2 = [host(b.solution(k)[0]) for k in range(3)]
    for a, c in zip(x1, x2):
        assert np.array_equal(a, c)
    b.close()


def test_batch_mixed_sizes_with_degenerate_instance():
    rng = np.random.default_rng(0)
    insts = [I.paper_example(1.0, 3.0, hi=50.0), I.tiny(), I.transit_instance(rng, 500),
             I.single_link([1.0, 2.0], [0, 1], 4.0, hi=50.0)]
    for i in insts:
        i.lo, i.hi = 0.0, 50.0
    b = BatchSolver(insts, dtype=torch.float64)
    res = b.solve(20000)
    for k, inst in enumerate(insts):
        o = oracle.run(inst, 100000, stop=True)
        xb, _, _ = b.solution(k)
        assert res[k]["converged"] and res[k]["iterations"] == o["iterations"]
        assert close(host(xb), o["x"], 64)
    b.close()


def test_stream_reordering_keeps_results():
    """Renumbering streams by their first link changes only where they live
    on the device, not any sum: results are identical and come back in the
    caller's numbering."""
    insts = _small_batch(count=4, seed=11)
    outs = []
    for reorder in (0, 1):
        b = BatchSolver(insts, dtype=torch.float32, eps_abs=0.0,
                        options=batch_options_default(reorder_streams=reorder))
        b.solve(70)
        outs.append([tuple(host(t) for t in b.solution(k)) for k in range(len(insts))])
        b.close()
    for (x0, l0, s0), (x1, l1, s1) in zip(*outs):
        assert np.array_equal(x0, x1) and np.array_equal(l0, l1) and np.array_equal(s0, s1)


def test_batch_with_alpha2_instance():
    a = I.tiny(seed=4)
    a.utility = np.random.default_rng(4).integers(0, 3, a.n).astype(np.uint8)
    insts = [a] + _small_batch(count=2)
    for i in insts:
        i.lo, i.hi = 0.0, float(max(i.hi, 10.0))
    b = BatchSolver(insts, dtype=torch.float64, eps_abs=0.0)
    b.solve(150)
    for k, inst in enumerate(insts):
        o = oracle.run(inst, 150)
        xb, lb, _ = b.solution(k)
        assert close(host(xb), o["x"], 64) and close(host(lb), o["lam"], 64)
    b.close()


def test_profile_phases_add_up():
    """The kernel's phase clocks (pmp_batch_profile) add up to about the
    duration of the solve, and profiling changes no result."""
    import time
    insts = [i.rounded(np.float32) for i in _small_batch(count=8, scale=0.05, seed=5)]
    outs = []
    for profile in (0, 1):
        b = BatchSolver(insts, dtype=torch.float32,
                        options=batch_options_default(profile=profile))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = b.solve(400)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        outs.append(([r["iterations"] for r in res],
                     [tuple(host(t) for t in b.solution(k)) for k in range(len(insts))]))
        if profile:
            ph = b.profile()
            total = sum(ph.values())
            print(f"phases {ph}, sum {total:.2f} ms, solve {dt * 1e3:.2f} ms", flush=True)
            assert all(v >= 0.0 for v in ph.values())
            assert 0.5 * dt * 1e3 <= total <= 1.05 * dt * 1e3
        b.close()
    assert outs[0][0] == outs[1][0]
    for (x0, l0, s0), (x1, l1, s1) in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(x0, x1) and np.array_equal(l0, l1) and np.array_equal(s0, s1)


def test_batch_results_independent_of_instance_order():
    """Stress: the same instances in a shuffled order give each instance the
    same iterations and iterates bit for bit (every sum stays inside its
    instance and tile)."""
    insts = [i.rounded(np.float32) for i in _small_batch(count=10, scale=0.02, seed=9)]
    perm = np.random.default_rng(1).permutation(len(insts))
    runs = []
    for order in (np.arange(len(insts)), perm):
        b = BatchSolver([insts[k] for k in order], dtype=torch.float32)
        res = b.solve(20000)
        got = {}
        for pos, k in enumerate(order):
            x, lam, _ = b.solution(pos)
            got[int(k)] = (res[pos]["iterations"], host(x), host(lam))
        b.close()
        runs.append(got)
    for k in range(len(insts)):
        a, c = runs[0][k], runs[1][k]
        assert a[0] == c[0] and np.array_equal(a[1], c[1]) and np.array_equal(a[2], c[2])
