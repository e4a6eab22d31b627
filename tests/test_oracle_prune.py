"""Pins of the oracle's link-failure pruning (Section V-D) on the CPU."""
import numpy as np
import pytest

from oracle import prune as orc_prune
from paper_2509_10722_amd import instances


def _dense(m, n, row_ptr, col_idx):
    R = np.zeros((m, n), np.int8)
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    R[rows, col_idx] = 1
    return R


def test_paper_example_by_hand():
    # Section III-A's network: link 1 -> stream 1; link 2 -> streams 2, 3;
    # link 3 -> streams 2, 4.  Link 2 fails: streams 2 and 3 lose their path,
    # links 1 and 3 remain with streams 1 and 4.
    inst = instances.paper_example()
    p = orc_prune.prune(inst, np.array([0, 1, 0], np.uint8))
    assert (p["m"], p["n"], p["nnz"]) == (2, 2, 2)
    assert p["row_ptr"].tolist() == [0, 1, 2]
    assert p["col_idx"].tolist() == [0, 1]
    assert p["link_map"].tolist() == [0, 2]
    assert p["stream_map"].tolist() == [0, 3]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_submatrix_and_route_invariants(seed):
    inst = instances.tiny(seed=seed)
    rng = np.random.default_rng(100 + seed)
    failed = (rng.random(inst.m) < 0.1).astype(np.uint8)
    p = orc_prune.prune(inst, failed)
    R = _dense(inst.m, inst.n, inst.row_ptr, inst.col_idx)
    Rp = _dense(p["m"], p["n"], p["row_ptr"], p["col_idx"])
    # the pruned pattern is the submatrix on the kept links and streams
    assert np.array_equal(Rp, R[np.ix_(p["link_map"], p["stream_map"])])
    # a stream is dropped exactly when its route crosses a failed link
    crosses = (R[failed.astype(bool)].sum(axis=0) > 0)
    assert np.array_equal(np.flatnonzero(~crosses), p["stream_map"])
    assert np.array_equal(np.flatnonzero(failed == 0), p["link_map"])
    # kept routes are whole, rows sorted
    assert np.array_equal(Rp.sum(axis=0), R[:, p["stream_map"]].sum(axis=0))
    for l in range(p["m"]):
        seg = p["col_idx"][p["row_ptr"][l]:p["row_ptr"][l + 1]]
        assert np.all(np.diff(seg) > 0)
    assert np.array_equal(p["c"], inst.c[p["link_map"]])
    assert np.array_equal(p["w"], inst.w[p["stream_map"]])


def test_no_failure_is_identity_and_all_fail_is_empty():
    inst = instances.tiny(seed=3)
    p = orc_prune.prune(inst, np.zeros(inst.m, np.uint8))
    assert np.array_equal(p["row_ptr"], inst.row_ptr)
    assert np.array_equal(p["col_idx"], inst.col_idx)
    q = orc_prune.prune(inst, np.ones(inst.m, np.uint8))
    assert (q["m"], q["n"], q["nnz"]) == (0, 0, 0)
    assert q["row_ptr"].tolist() == [0]
