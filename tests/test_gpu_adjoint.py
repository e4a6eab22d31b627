"""Reverse mode of K unrolled PMP iterations (pmp_forward_ckpt / pmp_backward).

Pins: (i) PyTorch autograd (FP64, CPU) over an independent dense re-statement
of the printed compact updates; (ii) central finite differences of the FP64
CPU oracle; (iii) the envelope relations dU*/dc = lambda and
dU*/dw_j = log x_j* at large K (KKT of Section VI-B).
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import optimality as opt
from paper_2509_10722_amd import instances as I
from tests.gpu_util import host, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2509_10722_amd.pmp import PMP_LAYOUT_BINNED, Solver, pmp_objective  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _utility_sum(inst, x):
    log = inst.utility == 0
    return float(np.sum(inst.w[log] * np.log(x[log])) + np.sum(inst.w[~log] * x[~log]))


def _torch_unrolled(inst, c, w, K, alpha=1.6, rho=1.0):
    """Dense FP64 torch restatement of the over-relaxed compact PMP updates."""
    m, n = inst.m, inst.n
    R = torch.zeros(m, n, dtype=torch.float64)
    rows = np.repeat(np.arange(m), np.diff(inst.row_ptr))
    R[rows, inst.col_idx] = 1.0
    L = R.sum(0)
    d = R.sum(1)
    log = torch.as_tensor(inst.utility == 0)
    a = torch.zeros(n, dtype=torch.float64)
    b = torch.zeros(m, dtype=torch.float64)
    zs = torch.zeros(m, dtype=torch.float64)
    u = torch.zeros(m, dtype=torch.float64)
    for _ in range(K):
        S = L * a + R.T @ (b - u)
        q = torch.sqrt(S * S + 4 * w * L / rho)
        xlog = torch.where(S >= 0, (S + q) / (2 * L), 2 * w / (rho * (q - S)))
        xlin = (S + w / rho) / L
        x = torch.clamp(torch.where(log, xlog, xlin), inst.lo, inst.hi)
        a = alpha * x + (1 - alpha) * a
        y = R @ x
        ps = torch.maximum(zs - u, -c)
        pbar = (y + ps) / (d + 1)
        b = -alpha * pbar + (1 - alpha) * b
        zs = alpha * (ps - pbar) + (1 - alpha) * zs
        u = u + alpha * pbar
    # separate sums: a where() over both branches would send log(0) of clipped
    # linear rates into the gradient as NaN
    J = torch.sum(w[log] * torch.log(x[log])) + torch.sum(w[~log] * x[~log])
    return J, x


@pytest.mark.parametrize("K,s", [(40, 7), (60, 60), (25, 1)])
def test_adjoint_matches_autograd_fp64(K, s):
    inst = I.tiny(scale=0.25)
    solver = Solver(inst, dtype=torch.float64, adapt_every=0)
    J = solver.forward_ckpt(K, s)
    gc, gw = solver.backward()
    c = torch.tensor(inst.c, requires_grad=True)
    w = torch.tensor(inst.w, requires_grad=True)
    Jt, _ = _torch_unrolled(inst, c, w, K)
    Jt.backward()
    print(f"K={K} s={s}: J {J:.12g} vs {Jt.item():.12g}; "
          f"dc {rel(host(gc), c.grad.numpy()):.2e} dw {rel(host(gw), w.grad.numpy()):.2e}")
    assert abs(J - Jt.item()) <= 1e-10 * abs(Jt.item())
    assert rel(host(gc), c.grad.numpy()) <= 1e-9
    assert rel(host(gw), w.grad.numpy()) <= 1e-9
    # the handle is back at iteration K
    x, _, _ = solver.solution()
    _, xt = _torch_unrolled(inst, c.detach(), w.detach(), K)
    assert rel(host(x), xt.numpy()) <= 1e-10
    solver.close()


def test_adjoint_directional_fd_of_oracle():
    inst = I.tiny()
    K = 150
    solver = Solver(inst, dtype=torch.float64, adapt_every=0)
    solver.forward_ckpt(K, 25)
    gc, gw = solver.backward()
    solver.close()
    rng = np.random.default_rng(3)
    dc = rng.normal(size=inst.m)
    dw = rng.normal(size=inst.n)
    h = 1e-6

    def J_at(t):
        p = I.Instance(inst.name, inst.m, inst.n, inst.row_ptr, inst.col_idx,
                       inst.c + t * dc, inst.w + t * dw, inst.utility, inst.lo, inst.hi)
        return _utility_sum(p, oracle.run(p, K, adapt_every=0)["x"])

    fd = (J_at(h) - J_at(-h)) / (2 * h)
    an = float(host(gc) @ dc + host(gw) @ dw)
    print(f"directional derivative: adjoint {an:.10g}, central FD {fd:.10g}")
    assert abs(an - fd) <= 1e-5 * max(1.0, abs(fd))


def test_envelope_relations_at_large_K():
    """dJ/dc -> lambda* and dJ/dw_j -> log x_j* (log streams) as K grows."""
    inst = I.single_link([0.5, 1.0, 1.7, 2.0], [0, 0, 0, 0], 6.0, hi=1e3)
    solver = Solver(inst, dtype=torch.float64, adapt_every=0)
    solver.forward_ckpt(3000, 100)
    gc, gw = solver.backward()
    solver.close()
    x_star = np.array([0.5, 1.0, 1.7, 2.0]) * 6.0 / 5.2
    lam_star = 5.2 / 6.0
    print("envelope: dc", host(gc), "lambda*", lam_star, "dw", host(gw), "log x*", np.log(x_star))
    assert abs(host(gc)[0] - lam_star) <= 1e-4 * lam_star
    np.testing.assert_allclose(host(gw), np.log(x_star), rtol=1e-4, atol=1e-6)


def test_envelope_tiny_reported():
    inst = I.tiny()
    solver = Solver(inst, dtype=torch.float64, adapt_every=0)
    solver.forward_ckpt(3000, 100)
    gc, gw = solver.backward()
    _, lam, _ = solver.solution()
    solver.close()
    o = oracle.run(inst, 100000, eps_abs=1e-10, stop=True, adapt_every=0)
    ec = rel(host(gc), o["lam"])
    print(f"tiny K=3000: ||dJ/dc - lambda*|| / ||lambda*|| = {ec:.2e}")
    assert ec < 5e-2


def test_adjoint_edge_shapes_fp64():
    """Reverse mode on ragged shapes (a route of 5000 links and a link on
    4500 streams, longer than one workgroup's stage; unused links; a stream
    with an empty route), FP64, in both layouts.  Exact pins: the empty-route
    stream's rate is hi whatever its weight, so dJ/dw there is U_j'(w) at
    x = hi (log hi or hi), and a capacity no stream crosses cannot move any
    rate, so dJ/dc is 0 there.  Then the two layouts against each other, and
    the directional derivative against a central difference of the oracle
    whose +h and -h runs took the prox branches of the unperturbed run in
    every iteration (branch digest): with 9000 rates over 100 iterations a
    step of 1e-6 already crosses a clip.  The oracle's J after 100 FP64
    iterations moves by about 1e-13 |J| under rounding (the scatter of
    kink-free differences between h = 5e-8 and 4e-7), so a difference at step
    h carries about 1e-13 |J| / h; the gate is 4x that plus 1e-6 relative."""
    inst = I.edge_shapes()
    K, s = 100, 25
    grads = {}
    for layout, name in ((1, "gather"), (2, "binned")):
        print(f"edge shapes: forward_ckpt({K}, {s}) + backward, FP64 {name}", flush=True)
        solver = Solver(inst, dtype=torch.float64, adapt_every=0, layout=layout)
        assert solver.layout_in_use() == name
        solver.forward_ckpt(K, s)
        gc, gw = solver.backward()
        solver.close()
        grads[name] = (host(gc), host(gw))
    gc, gw = grads["gather"]
    j = inst.n - 1
    assert gw[j] == (np.log(inst.hi) if inst.utility[j] == 0 else inst.hi)
    unused = np.flatnonzero(np.diff(inst.row_ptr) == 0)
    assert unused.size >= 5 and np.all(gc[unused] == 0.0)
    for k in range(2):
        assert rel(grads["binned"][k], grads["gather"][k]) <= 1e-10
    rng = np.random.default_rng(5)
    dc = rng.normal(size=inst.m)
    dw = rng.normal(size=inst.n)

    def J_at(t):
        p = I.Instance(inst.name, inst.m, inst.n, inst.row_ptr, inst.col_idx,
                       inst.c + t * dc, inst.w + t * dw, inst.utility, inst.lo, inst.hi)
        o = oracle.run(p, K, adapt_every=0, branches=True)
        return _utility_sum(p, o["x"]), o["branch_digest"]

    J0, d0 = J_at(0.0)
    for h in (4e-7, 2e-7, 1e-7):
        (jp, dp), (jm, dm) = J_at(h), J_at(-h)
        if dp == d0 and dm == d0:
            break
    else:
        pytest.fail("every step crossed a prox kink")
    fd = (jp - jm) / (2 * h)
    tol = 1e-6 * abs(fd) + 4.0 * 1e-13 * abs(J0) / h
    an = float(gc @ dc + gw @ dw)
    print(f"  directional derivative: adjoint {an:.10g}, central FD (h={h:g}) {fd:.10g}, "
          f"|diff| / tol {abs(an - fd) / tol:.3f}", flush=True)
    assert abs(an - fd) <= tol


def test_autograd_function_fp32():
    inst = I.tiny().rounded(np.float32)
    solver = Solver(inst, dtype=torch.float32, adapt_every=0)
    c = torch.tensor(inst.c, dtype=torch.float32, device="cuda", requires_grad=True)
    w = torch.tensor(inst.w, dtype=torch.float32, device="cuda", requires_grad=True)
    J = pmp_objective(c, w, solver, 200, 20)
    J.backward()
    ref = Solver(inst, dtype=torch.float64, adapt_every=0)
    ref.forward_ckpt(200, 20)
    gc64, gw64 = ref.backward()
    solver.close(); ref.close()
    assert rel(host(c.grad), host(gc64)) <= 1e-4
    assert rel(host(w.grad), host(gw64)) <= 1e-4


def test_adjoint_alpha2_directional_fd():
    inst = I.tiny(seed=9)
    rng = np.random.default_rng(9)
    inst.utility = rng.integers(0, 3, inst.n).astype(np.uint8)
    K = 120
    solver = Solver(inst, dtype=torch.float64, adapt_every=0)
    solver.forward_ckpt(K, 16)
    gc, gw = solver.backward()
    solver.close()
    dc = rng.normal(size=inst.m)
    dw = rng.normal(size=inst.n)
    h = 1e-6

    def J_at(t):
        p = I.Instance(inst.name, inst.m, inst.n, inst.row_ptr, inst.col_idx,
                       inst.c + t * dc, inst.w + t * dw, inst.utility, inst.lo, inst.hi)
        x = oracle.run(p, K, adapt_every=0)["x"]
        return opt.utility(p, x)

    fd = (J_at(h) - J_at(-h)) / (2 * h)
    an = float(host(gc) @ dc + host(gw) @ dw)
    print(f"alpha2 directional derivative: adjoint {an:.10g}, FD {fd:.10g}")
    assert abs(an - fd) <= 1e-5 * max(1.0, abs(fd))


def _golden_fd(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _fd_tol(fd, trunc, scale):
    """Tolerance of an FP32 gradient entry against an FP64 central difference:
    8x the difference's truncation error (estimated from its 2h repeat), 1e-5
    relative for the FP32 rounding of the unrolled iterates carried into the
    gradient (1e-6 normwise on the iterates after 500 iterations, tens of
    eps32 on single entries), and an absolute floor of 1e-6 of the typical
    entry for gradients near zero."""
    return 8.0 * trunc + 1e-5 * abs(fd) + 1e-6 * scale


def _direction_check(an, d, h):
    """Directional derivative against the oracle's central difference with
    the largest step (1e-3, 1e-5, 1e-7) whose +h and -h runs took the same
    prox branches in every iteration (branch digest).  Along a direction every
    coordinate moves, so with a large step some clip or slack branch changes
    inside the interval and the difference is the mean slope across kinks,
    not the derivative (on the full workload h = 1e-3 gives -40.6 and 1e-5
    -37.5 against a derivative of -36.90).  Tolerance: 2e-5 relative for the
    FP32 iterates, 8x the step's truncation estimate where there is one, and
    4x its FD64 rounding eps |J| / h.  Returns (passed, tolerance, step)."""
    steps = [dict(h=h, fd=d["fd"], branch_flip=d["branch_flip"], trunc=d["trunc"],
                  rounding=0.0)] + d["small_steps"]
    usable = [st for st in steps if not st["branch_flip"]]
    assert usable, "every step crossed a prox kink"
    st = usable[0]
    tol = 2e-5 * abs(st["fd"]) + 8.0 * st.get("trunc", 0.0) + 4.0 * st["rounding"]
    return abs(an - st["fd"]) <= tol, tol, st


def test_adjoint_workload_fp32_binned_vs_oracle_fd():
    """Pattern 3 at its own configuration: FP32, binned layout, K = 500 with
    checkpoints every s = 25, fixed rho = 1, on the adjoint workload at scale
    0.1 (m = 1e4, n = 1e5), against central differences (h = 1e-3) of the
    FP64 oracle for 32 capacities, 32 weights and one random direction
    (tests/golden/make_adjoint_fd.py).  Pairs whose +h and -h runs took
    different prox branches are skipped (not a derivative there).  The
    distance of dJ/dc to the converged prices lambda* (envelope, Section
    VI-B) is reported: at K = 500 the iterate is far from converged."""
    g = _golden_fd("adjoint_fd.json")
    inst = I.adjoint(scale=0.1).rounded(np.float32)
    assert f"m={inst.m}, n={inst.n}, nnz={inst.nnz}" in g["workload"]
    print(f"adjoint scale 0.1: forward_ckpt({g['K']}, 25) + backward, FP32 binned", flush=True)
    solver = Solver(inst, dtype=torch.float32, adapt_every=0, layout=PMP_LAYOUT_BINNED)
    assert solver.layout_in_use() == "binned"
    J = solver.forward_ckpt(g["K"], 25)
    gc, gw = solver.backward()
    solver.close()
    gc, gw = host(gc), host(gw)
    assert abs(J - g["J"]) <= 1e-6 * abs(g["J"])
    rng = np.random.default_rng(g["seed"])
    links = np.sort(rng.choice(inst.m, len(g["links"]), replace=False))
    streams = np.sort(rng.choice(inst.n, len(g["streams"]), replace=False))
    dc = rng.normal(size=inst.m)
    dw = rng.normal(size=inst.n)
    assert [r["index"] for r in g["links"]] == links.tolist()
    assert [r["index"] for r in g["streams"]] == streams.tolist()
    checked, worst = 0, 0.0
    for grad, rows in ((gc, g["links"]), (gw, g["streams"])):
        scale = np.sqrt(np.mean([r["fd"] ** 2 for r in rows]))
        for r in rows:
            if r["branch_flip"]:
                continue
            gi = float(grad[r["index"]])
            tol = _fd_tol(r["fd"], r["trunc"], scale)
            worst = max(worst, abs(gi - r["fd"]) / tol)
            assert abs(gi - r["fd"]) <= tol, (r, gi)
            checked += 1
    d = g["direction"]
    an = float(gc @ dc + gw @ dw)
    lam_at = np.array(g["lambda_star"]["at_links"])
    env = np.abs(gc[links] - lam_at) / np.maximum(np.abs(lam_at), 1e-12)
    ok, tol, st = _direction_check(an, d, g["h"])
    print(f"  {checked} of {len(g['links']) + len(g['streams'])} coordinates checked, worst "
          f"|grad - fd| / tol {worst:.3f}; direction: adjoint {an:.10g}, FD h={st['h']:g} "
          f"{st['fd']:.10g} (|diff| / tol {abs(an - st['fd']) / tol:.3f}; h=1e-3 gave "
          f"{d['fd']:.10g}); envelope: "
          f"||dJ/dc|| {np.linalg.norm(gc):.4g} vs ||lambda*|| {g['lambda_star']['norm']:.4g}, "
          f"sampled |dJ/dc - lambda*| / lambda* median {np.median(env):.3f} max {np.max(env):.3f}")
    assert checked >= 48
    assert ok


def test_adjoint_full_workload_directional_fd():
    """The benchmarked configuration itself (scale 1: m = 1e5, n = 1e6, FP32,
    binned, K = 500, s = 25): the directional derivative along one random
    direction against the oracle's central differences (see
    _direction_check)."""
    g = _golden_fd("adjoint_fd_scale1.json")
    inst = I.adjoint(scale=1.0).rounded(np.float32)
    assert f"m={inst.m}, n={inst.n}, nnz={inst.nnz}" in g["workload"]
    print(f"adjoint scale 1: forward_ckpt({g['K']}, 25) + backward, FP32 binned", flush=True)
    solver = Solver(inst, dtype=torch.float32, adapt_every=0)
    assert solver.layout_in_use() == "binned"
    J = solver.forward_ckpt(g["K"], 25)
    gc, gw = solver.backward()
    solver.close()
    rng = np.random.default_rng(g["seed"])
    rng.choice(inst.m, 0, replace=False)
    rng.choice(inst.n, 0, replace=False)
    dc = rng.normal(size=inst.m)
    dw = rng.normal(size=inst.n)
    an = float(host(gc) @ dc + host(gw) @ dw)
    d = g["direction"]
    ok, tol, st = _direction_check(an, d, g["h"])
    print(f"  J {J:.10g} (oracle {g['J']:.10g}); direction: adjoint {an:.10g}, FD h={st['h']:g} "
          f"{st['fd']:.10g} (|diff| / tol {abs(an - st['fd']) / tol:.3f}; h=1e-3 gave "
          f"{d['fd']:.10g})")
    assert abs(J - g["J"]) <= 1e-6 * abs(g["J"])
    assert ok
