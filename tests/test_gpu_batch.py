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
    for caps in ((64, 64, 64), (8192, 8192, 8192), (512, 1024, 2048), (4096, 8192, 4096)):
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


@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_batch_edge_shapes_match_plain_gather_solves(dtype_name):
    """Ragged shapes inside a batch, next to an ordinary instance: a route of
    5000 links (a stream tile of its own, summed strided) and a link on 4500
    streams (a chunk tile), links no stream uses, a stream with an empty
    route (its rate is hi) and single-link streams.  The iterates equal the
    one-at-a-time gather solves bit for bit; in FP64 they also meet the
    oracle at equal iteration count."""
    dtype = getattr(torch, dtype_name)
    insts = [I.edge_shapes(), I.tiny()]
    if dtype_name == "float32":
        insts = [i.rounded(np.float32) for i in insts]
    K = 300
    print(f"edge shapes in a batch, {dtype_name}, {K} iterations", flush=True)
    b = BatchSolver(insts, dtype=dtype, eps_abs=0.0)
    res = b.solve(K)
    for k, inst in enumerate(insts):
        s = Solver(inst, dtype=dtype, layout=1, eps_abs=0.0, max_iter=K)
        r = s.solve()
        x, lam, _ = s.solution()
        xb, lb, _ = b.solution(k)
        print(f"  instance {k} ({inst.name}): batch rho {res[k]['rho']}, plain rho {r['rho']}",
              flush=True)
        assert res[k]["iterations"] == r["iterations"] == K
        assert res[k]["rho"] == r["rho"]
        assert torch.equal(x, xb) and torch.equal(lam, lb)
        s.close()
    xe, le, _ = b.solution(0)
    xe, le = host(xe), host(le)
    assert xe[-1] == insts[0].hi
    if dtype_name == "float64":
        o = oracle.run(insts[0], K)
        assert close(xe, o["x"], 64) and close(le, o["lam"], 64)
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


def _congested_batch(dtype_name):
    """Two congested instances (Section V-C: 0.1% of the links on 10% of the
    streams; rows of 5,000 and 10,000 nonzeros) beside a transit instance."""
    insts = [I.congested(I.medium(scale=0.1), seed=6),
             I.batched(count=1, scale=0.01)[0],
             I.congested(I.medium(seed=7, scale=0.2), seed=9)]
    return [i.rounded(np.float32) for i in insts] if dtype_name == "float32" else insts


@pytest.mark.parametrize("dtype_name,chunk", [("float32", 1024), ("float32", 8192),
                                              ("float32", 1 << 20), ("float64", 8192)])
def test_congested_batch_matches_plain_gather_solves(dtype_name, chunk):
    """Long link rows in chunk tiles (heavy_chunk) finished by the last
    arriving workgroup: the iterates equal those of one-at-a-time solves in
    the gather layout bit for bit.  In FP32 (finite box) the long rows are
    exact fixed-point sums, so any chunk size gives them; in FP64 the 8192
    chunks are the gather layout's own."""
    dtype = getattr(torch, dtype_name)
    insts = _congested_batch(dtype_name)
    K = 300
    print(f"congested batch {dtype_name}, heavy_chunk {chunk}, {K} iterations", flush=True)
    b = BatchSolver(insts, dtype=dtype, eps_abs=0.0,
                    options=batch_options_default(heavy_chunk=chunk))
    res = b.solve(K)
    for k, inst in enumerate(insts):
        s = Solver(inst, dtype=dtype, layout=1, eps_abs=0.0, max_iter=K)
        r = s.solve()
        x, lam, _ = s.solution()
        xb, lb, _ = b.solution(k)
        deg = int(np.diff(inst.row_ptr).max())
        print(f"  instance {k} (m={inst.m}, longest row {deg}): batch rho {res[k]['rho']}, "
              f"plain rho {r['rho']}", flush=True)
        assert res[k]["iterations"] == r["iterations"] == K
        assert res[k]["rho"] == r["rho"]
        assert torch.equal(x, xb) and torch.equal(lam, lb)
        s.close()
    b.close()


def test_congested_batch_fp64_small_chunks_repeat():
    """FP64 long rows in chunks of 1024 (other chunk sums than the gather
    layout's): two solves from the same start agree bit for bit whatever
    workgroup arrives last, and stay within rounding of the plain solve."""
    insts = _congested_batch("float64")
    K = 200
    b = BatchSolver(insts, dtype=torch.float64, eps_abs=0.0,
                    options=batch_options_default(heavy_chunk=1024))
    runs = []
    for _ in range(2):
        b.reset()
        b.solve(K)
        runs.append([host(b.solution(k)[0]) for k in range(len(insts))])
    for a, c in zip(*runs):
        assert np.array_equal(a, c)
    for k, inst in enumerate(insts):
        s = Solver(inst, dtype=torch.float64, layout=1, eps_abs=0.0, max_iter=K)
        s.solve()
        x = host(s.solution()[0])
        s.close()
        assert np.max(np.abs(runs[0][k] - x)) <= 1e-9 * max(1.0, np.max(np.abs(x)))
    b.close()


def test_autotuner_heavy_row_class(tmp_path):
    """With congested instances present the tuner times the long-row chunk
    candidates and caches the choice (per architecture) next to the tile caps."""
    from paper_2509_10722_amd import autotune
    insts = _congested_batch("float32")
    path = str(tmp_path / "tiles.json")
    opts, timings = autotune.tune_batch(insts, dtype=torch.float32, iters=20, reps=1,
                                        candidates=(1024, 4096), heavy_candidates=(1024, 8192),
                                        path=path)
    print({k: round(v * 1e3, 3) for k, v in timings.items()}, flush=True)
    assert {"heavy:1024", "heavy:8192"} <= set(timings)
    assert autotune.cached_options(torch, path).heavy_chunk == opts.heavy_chunk in (1024, 8192)
    plain = autotune.tune_batch([I.batched(count=1, scale=0.01)[0]], dtype=torch.float32,
                                iters=10, reps=1, candidates=(4096,), path=path)[1]
    assert not any(k.startswith("heavy:") for k in plain)


def test_congested_batch_to_tolerance_matches_plain():
    """Solved to the 1e-4 rule, the instances stop at different checks (a
    stopped instance's chunk tiles are skipped while the others run on); every
    instance stops at the plain gather solve's iteration with its iterate bit
    for bit (FP32, fixed-point long rows, chunks of 1024)."""
    insts = _congested_batch("float32")
    b = BatchSolver(insts, dtype=torch.float32, options=batch_options_default(heavy_chunk=1024))
    res = b.solve(30000)
    its = []
    for k, inst in enumerate(insts):
        s = Solver(inst, dtype=torch.float32, layout=1, max_iter=30000)
        r = s.solve()
        x, lam, _ = s.solution()
        xb, lb, _ = b.solution(k)
        print(f"  instance {k}: batch {res[k]['iterations']} it, plain {r['iterations']} it", flush=True)
        assert res[k]["converged"] and r["converged"]
        assert res[k]["iterations"] == r["iterations"]
        assert torch.equal(x, xb) and torch.equal(lam, lb)
        its.append(r["iterations"])
        s.close()
    b.close()
    assert len(set(its)) > 1


def test_barrier_wait_bound_reports_error_and_gpu_recovers():
    """A grid barrier wait bounded at 2 polls (wait_log2 = 1) expires at once:
    every workgroup leaves the kernel, pmp_batch_solve returns PMP_ERR_HIP, and
    a batch set up afterwards with the default bound solves as usual."""
    from paper_2509_10722_amd.pmp import PMP_ERR_HIP, PMPError
    insts = [i.rounded(np.float32) for i in _small_batch(count=3)]
    print("batch with wait_log2 = 1 (forced barrier expiry)", flush=True)
    b = BatchSolver(insts, dtype=torch.float32, options=batch_options_default(wait_log2=1))
    with pytest.raises(PMPError) as e:
        b.solve(50)
    assert e.value.status == PMP_ERR_HIP
    b.close()
    print("batch with the default bound", flush=True)
    good = BatchSolver(insts, dtype=torch.float32)
    res = good.solve(20000)
    good.close()
    ref = BatchSolver(insts, dtype=torch.float32)
    res2 = ref.solve(20000)
    ref.close()
    assert all(r["converged"] for r in res)
    assert [r["iterations"] for r in res] == [r["iterations"] for r in res2]
