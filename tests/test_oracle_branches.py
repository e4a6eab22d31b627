"""The oracle's prox-branch digest (which clip and slack-projection branch
every prox took, over every iteration), used to discard finite-difference
pairs that straddle a kink of the iteration map."""
import numpy as np

import oracle
from paper_2509_10722_amd import instances as I


def _with(inst, c=None, w=None):
    return I.Instance(inst.name, inst.m, inst.n, inst.row_ptr, inst.col_idx,
                      inst.c if c is None else c, inst.w if w is None else w,
                      inst.utility, inst.lo, inst.hi)


def test_digest_is_deterministic_and_thread_independent():
    inst = I.tiny()
    a = oracle.run(inst, 200, branches=True, threads=1)
    b = oracle.run(inst, 200, branches=True, threads=4)
    assert a["branch_digest"] == b["branch_digest"] != 0
    assert np.array_equal(a["x"], b["x"])
    assert "branch_digest" not in oracle.run(inst, 5)


def test_digest_tracks_branches_only():
    inst = I.tiny()
    base = oracle.run(inst, 200, adapt_every=0, branches=True)["branch_digest"]
    # a tiny smooth change of one weight moves x but no branch
    w = inst.w.copy()
    w[3] *= 1 + 1e-12
    o = oracle.run(_with(inst, w=w), 200, adapt_every=0, branches=True)
    assert o["branch_digest"] == base
    # halving every capacity makes other links tight (slack projected) and
    # other rates clip
    o = oracle.run(_with(inst, c=inst.c * 0.5), 200, adapt_every=0, branches=True)
    assert o["branch_digest"] != base


def test_digest_sees_a_single_slack_branch():
    """One link carrying one log stream: with c = 1 the link binds during
    the run, with c = 1e5 it stays far from its capacity, so the slack
    branches differ and so do the digests."""
    tight = I.single_link([1.0], [0], 1.0, hi=1e6)
    loose = I.single_link([1.0], [0], 1e5, hi=1e6)
    a = oracle.run(tight, 50, adapt_every=0, branches=True)["branch_digest"]
    b = oracle.run(loose, 50, adapt_every=0, branches=True)["branch_digest"]
    assert a != b
