"""Generator checks: shapes, distinct links per route, distributions, seeds."""
import numpy as np

from paper_2509_10722_amd import instances as I


def _check_pattern(inst):
    assert inst.row_ptr.dtype == np.int32 and inst.col_idx.dtype == np.int32
    assert inst.row_ptr[0] == 0 and inst.row_ptr[-1] == inst.col_idx.size
    assert np.all(np.diff(inst.row_ptr) >= 0)
    assert inst.col_idx.min() >= 0 and inst.col_idx.max() < inst.n
    for l in range(inst.m):
        row = inst.col_idx[inst.row_ptr[l]:inst.row_ptr[l + 1]]
        assert np.all(np.diff(row) > 0)           # sorted, unique => 0/1


def test_tiny_recipe():
    t = I.tiny()
    _check_pattern(t)
    L = np.bincount(t.col_idx, minlength=t.n)
    assert L.min() >= 2 and L.max() <= 8
    assert t.m == 200 and t.n == 1000
    assert np.all((t.c >= 1) & (t.c <= 10))
    assert (t.utility == I.LOG).sum() == 500
    assert np.all((t.w[t.utility == I.LOG] >= 0.5) & (t.w[t.utility == I.LOG] <= 2))
    assert np.all((t.w[t.utility == I.LINEAR] >= 0.1) & (t.w[t.utility == I.LINEAR] <= 1))
    assert t.lo == 0.0 and t.hi == 10.0


def test_seed_reproducible():
    a, b = I.tiny(), I.tiny()
    assert np.array_equal(a.col_idx, b.col_idx) and np.array_equal(a.c, b.c)
    c = I.tiny(seed=7)
    assert not np.array_equal(a.col_idx, c.col_idx)


def test_large_shape_scaled():
    t = I.large(scale=0.002)
    _check_pattern(t)
    L = np.bincount(t.col_idx, minlength=t.n)
    assert L.min() >= 3 and L.max() <= 40
    # discrete power law alpha=2.5 on 3..40 has mean 5.83
    assert abs(L.mean() - 5.83) < 0.2
    assert np.all(t.utility == I.LOG)


def test_transit_routes_are_diagonals():
    rng = np.random.default_rng(0)
    t = I.transit_instance(rng, 2000)
    _check_pattern(t)
    T = 48
    rows = np.repeat(np.arange(t.m), np.diff(t.row_ptr))
    order = np.lexsort((rows, t.col_idx))
    s, l = t.col_idx[order], rows[order]
    same = s[1:] == s[:-1]
    # consecutive links of a trip: next segment, next time bin
    assert np.all((l[1:] - l[:-1])[same] == T + 1)


def test_block_diagonal():
    a = I.paper_example()
    b = I.single_link([1.0, 2.0], [0, 0], 3.0)
    u = I.block_diagonal([a, b])
    _check_pattern(u)
    assert u.m == 4 and u.n == 6 and u.nnz == 7


def test_congested_adds_dense_rows():
    base = I.medium(scale=0.05)
    c = I.congested(base, link_frac=0.002, stream_frac=0.1)
    _check_pattern(c)
    deg = np.diff(c.row_ptr)
    hot = np.argsort(deg)[-10:]
    assert deg[hot].min() >= 0.1 * base.n * 0.99
    assert c.nnz > base.nnz
    # every original pair is still there
    rows = np.repeat(np.arange(base.m), np.diff(base.row_ptr))
    rows_c = np.repeat(np.arange(c.m), np.diff(c.row_ptr))
    orig = set((rows * base.n + base.col_idx).tolist())
    assert orig <= set((rows_c * c.n + c.col_idx).tolist())


def test_transit_case_study_sizes_and_routes():
    inst, meta = I.transit_case_study()
    _check_pattern(inst)
    assert (inst.m, inst.n) == (182784, 19800)       # Section VI's sizes
    T, src, dst = meta["T"], meta["edge_src"], meta["edge_dst"]
    assert src.size * T == inst.m
    # each edge has its reverse; no self loops
    assert set(zip(src.tolist(), dst.tolist())) == set(zip(dst.tolist(), src.tolist()))
    assert np.all(src != dst)
    for (o, d), rs in zip(meta["od_pairs"], meta["routes"]):
        for r in rs:
            # a path from o to d along existing edges
            assert src[r[0]] == o and dst[r[-1]] == d
            assert all(dst[a] == src[b] for a, b in zip(r[:-1], r[1:]))
    # stream j uses (e_k, t0 + k) along its route, one time bin per edge
    rows = np.repeat(np.arange(inst.m), np.diff(inst.row_ptr))
    for j in (0, 1, 4321, inst.n - 1):
        links = np.sort(rows[inst.col_idx == j])
        r = meta["routes"][meta["od"][j]][meta["route"][j]]
        want = np.sort(np.asarray(r) * T + meta["t0"][j] + np.arange(len(r)))
        assert np.array_equal(links, want)
    assert np.all(inst.w == 1.0) and np.all(inst.utility == I.LOG)


def test_transit_case_study_small():
    inst, meta = I.transit_case_study(stations=12, T=16, edges=30, od_pairs=6, departures=4)
    _check_pattern(inst)
    assert inst.m == 30 * 16 and inst.n == 6 * 2 * 4


def test_heavy_row_class_detection():
    """The autotuner's heavy-row class: instances with a link row longer than
    4096 nonzeros (congested links at 10% of 5e4 streams), not plain ones."""
    from paper_2509_10722_amd import autotune
    base = I.medium(scale=0.1)
    assert not autotune.has_heavy_rows(base)
    assert autotune.has_heavy_rows(I.congested(base))
    assert not autotune.has_heavy_rows(I.congested(I.medium(scale=0.05)))   # rows of 2,500


def test_edge_shapes_recipe():
    """The ragged parity instance has what its docstring promises: a route
    and a link longer than 4096 entries, unused links, an empty route."""
    inst = I.edge_shapes()
    _check_pattern(inst)
    deg = np.diff(inst.row_ptr)
    L = np.bincount(inst.col_idx, minlength=inst.n)
    assert deg[inst.m - 1] == 4500 and deg.max() == 4500
    assert np.all(deg[inst.m - 10:inst.m - 1] == 0)
    assert L[0] == 5000 and L[inst.n - 1] == 0
    assert L[1:inst.n - 1].min() >= 1 and L[1:inst.n - 1].max() <= 4
    assert np.isfinite(inst.hi)
