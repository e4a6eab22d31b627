"""pmp_prune_noalloc: pmp_prune with its scratch in the library's fixed
per-device array instead of a caller workspace, for callers that cannot
allocate.  Its outputs must equal pmp_prune's bit for bit (the same kernels
on the same data), on two calls in a row with the second on a smaller
instance (the fixed array then holds the first call's contents)."""
import numpy as np
import pytest

from paper_2509_10722_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2509_10722_amd.pmp import PMP_ERR_SHAPE, PMPError, Solver  # noqa: E402


def _pruned(solver, failed, noalloc):
    p, link_map, stream_map = solver.prune(failed, noalloc=noalloc)
    ins = p.instance
    arrays = [ins.row_ptr, ins.col_idx, ins.c, ins.w, ins.utility, link_map, stream_map,
              p.get_state()]
    out = [t.detach().cpu().numpy().view(np.uint8).copy() for t in arrays]
    p.iterate(25)
    x, lam, _ = p.solution()
    out += [x.cpu().numpy().view(np.uint8).copy(), lam.cpu().numpy().view(np.uint8).copy()]
    sizes = (ins.m, ins.n, int(ins.row_ptr[-1].item()))
    p.close()
    return sizes, out


@pytest.mark.parametrize("order", ["large_then_small", "small_then_large"])
def test_noalloc_prune_equals_workspace_prune(order):
    cases = [("medium x0.2, FP32", I.medium(scale=0.2).rounded(np.float32), torch.float32, 0.10),
             ("tiny, FP64", I.tiny(), torch.float64, 0.25)]
    if order == "small_then_large":
        cases = cases[::-1]
    for name, inst, dtype, frac in cases:
        print(f"noalloc prune: {name} (m={inst.m}, n={inst.n})", flush=True)
        s = Solver(inst, dtype=dtype)
        s.iterate(40)
        failed = (np.random.default_rng(inst.m).random(inst.m) < frac).astype(np.uint8)
        sz_a, a = _pruned(s, failed, noalloc=True)
        sz_b, b = _pruned(s, failed, noalloc=False)
        s.close()
        assert sz_a == sz_b and sz_a[0] < inst.m
        for k, (u, v) in enumerate(zip(a, b)):
            assert np.array_equal(u, v), (name, k)


def test_noalloc_prune_rejects_more_than_its_scratch():
    inst = I.large(scale=0.1).rounded(np.float32)      # m + n = 2.5e6
    s = Solver(inst, dtype=torch.float32)
    with pytest.raises(PMPError) as e:
        s.prune(np.zeros(inst.m, np.uint8), noalloc=True)
    s.close()
    assert e.value.status == PMP_ERR_SHAPE and "fixed maximum" in str(e.value)
