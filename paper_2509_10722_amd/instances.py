"""Seeded synthetic NUM instances (inputs only).

This module draws problem data and nothing else: link-route patterns, link
capacities, stream weights and utility types.  It holds none of the solver's
arithmetic, so both the FP64 CPU oracle (test infrastructure) and the HIP path
take their inputs from here.

The paper's experiments are synthetic (Section V-B: random link-route matrices
with n = m/2 and an average route of 10 links; Section V-C: congestion; Section
VI: a time-expanded transit network).  The recipes below have the shapes of
those workloads:

  tiny     m=200, n=1000, route length U{2..8}, c~U[1,10], half log
           (w~U[0.5,2]) / half linear (w~U[0.1,1]), box [0,10]
  medium   m=1e5, n=5e5, route length U{4..16}, c~U[1,100], 70% log / 30%
           linear, box [0, max c]
  large    m=5e6, n=2e7, route length from a discrete power law P(L) ~ L^-2.5
           on {3..40}, c ~ lognormal(2, 1), all log w~U[0.5,2], box [0, max c]
  adjoint  m=1e5, n=1e6, route length U{3..12}, all log, c~U[1,100]
  paper    the scaling shape of Section V-B: n=m/2, route length U{5..15}
  batched  64 transit-style instances (line network x 48 time bins, trips on
           consecutive segment-time links), capacities degraded on 10% of links
  transit_case_study  Section VI's time-expanded network at its sizes:
           100 stations, 952 directed edges x 192 bins = 182,784 links,
           110 OD pairs x 2 routes x 90 departures = 19,800 streams, w = 1

Every route consists of distinct links (R is a 0/1 matrix, eq. (1)).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

LOG = 0
LINEAR = 1
ALPHA2 = 2      # -w / x, minimum potential delay fairness


@dataclasses.dataclass
class Instance:
    """One NUM instance: maximize sum U_j(x_j) s.t. R x <= c, lo <= x <= hi.

    R (m x n, 0/1) is given by its CSR pattern: row_ptr[m+1], col_idx[nnz]
    (int32, sorted and unique within each row).  c[m] > 0, w[n] > 0 and
    utility[n] in {LOG, LINEAR} (uint8).
    """
    name: str
    m: int
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    c: np.ndarray
    w: np.ndarray
    utility: np.ndarray
    lo: float = 0.0
    hi: float = math.inf

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def rounded(self, dtype) -> "Instance":
        """Copy whose c and w are rounded to `dtype` and held again as float64.

        A parity comparison between an FP32 solver and the FP64 oracle must
        solve the same problem, so both receive the FP32-representable data.
        """
        return dataclasses.replace(
            self,
            c=self.c.astype(dtype).astype(np.float64),
            w=self.w.astype(dtype).astype(np.float64))

    def stats(self) -> dict:
        deg = np.diff(self.row_ptr)
        L = np.bincount(self.col_idx, minlength=self.n)
        return {"m": self.m, "n": self.n, "nnz": self.nnz,
                "route_len_mean": float(L.mean()) if self.n else 0.0,
                "route_len_max": int(L.max()) if self.n else 0,
                "link_deg_mean": float(deg.mean()) if self.m else 0.0,
                "link_deg_max": int(deg.max()) if self.m else 0,
                "log_fraction": float((self.utility == LOG).mean()) if self.n else 0.0}


def csr_from_pairs(m: int, n: int, link: np.ndarray, stream: np.ndarray):
    """CSR (row_ptr, col_idx) of the 0/1 matrix with ones at (link, stream)."""
    key = np.sort(link.astype(np.int64) * n + stream.astype(np.int64))
    rows = key // n
    cols = (key - rows * n).astype(np.int32)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    return row_ptr.astype(np.int32), cols


def random_routes(rng: np.random.Generator, m: int, lengths: np.ndarray):
    """Routes of the given lengths, each a set of distinct links drawn uniformly.

    Returns (link, stream) pairs, one per nonzero of R.
    """
    n = lengths.size
    L = lengths.astype(np.int64)
    if np.any(L > m):
        raise ValueError("route longer than the number of links")
    stream = np.repeat(np.arange(n, dtype=np.int64), L)
    link = rng.integers(0, m, stream.size, dtype=np.int64)
    while True:
        key = np.sort(stream * m + link)
        stream = key // m
        link = key - stream * m
        dup = np.flatnonzero(key[1:] == key[:-1]) + 1
        if dup.size == 0:
            return link, stream
        link[dup] = rng.integers(0, m, dup.size, dtype=np.int64)


def power_law_lengths(rng, n, alpha, lmin, lmax):
    vals = np.arange(lmin, lmax + 1)
    p = vals.astype(np.float64) ** (-alpha)
    p /= p.sum()
    return rng.choice(vals, size=n, p=p)


def _mixed_utilities(rng, n, log_fraction):
    perm = rng.permutation(n)
    utility = np.full(n, LINEAR, dtype=np.uint8)
    utility[perm[: int(round(log_fraction * n))]] = LOG
    w = np.where(utility == LOG, rng.uniform(0.5, 2.0, n), rng.uniform(0.1, 1.0, n))
    return utility, w


def random_instance(name, seed, m, n, lengths_fn, cap_fn, log_fraction, hi=None):
    rng = np.random.default_rng(seed)
    lengths = lengths_fn(rng, n)
    link, stream = random_routes(rng, m, lengths)
    row_ptr, col_idx = csr_from_pairs(m, n, link, stream)
    del link, stream
    c = cap_fn(rng, m)
    utility, w = _mixed_utilities(rng, n, log_fraction)
    hi_v = float(c.max()) if hi is None else float(hi)
    return Instance(name, m, n, row_ptr, col_idx, c, w, utility, 0.0, hi_v)


def tiny(seed=0, scale=1.0):
    m, n = max(8, int(200 * scale)), max(8, int(1000 * scale))
    return random_instance("tiny", seed, m, n,
                           lambda r, k: r.integers(2, 9, k),
                           lambda r, k: r.uniform(1.0, 10.0, k), 0.5, hi=10.0)


def medium(seed=1, scale=1.0):
    m, n = max(16, int(1e5 * scale)), max(16, int(5e5 * scale))
    return random_instance("medium", seed, m, n,
                           lambda r, k: r.integers(4, 17, k),
                           lambda r, k: r.uniform(1.0, 100.0, k), 0.7)


def large(seed=2, scale=1.0):
    m, n = max(64, int(5e6 * scale)), max(64, int(2e7 * scale))
    return random_instance("large", seed, m, n,
                           lambda r, k: power_law_lengths(r, k, 2.5, 3, 40),
                           lambda r, k: r.lognormal(2.0, 1.0, k), 1.0)


def adjoint(seed=4, scale=1.0):
    m, n = max(16, int(1e5 * scale)), max(16, int(1e6 * scale))
    return random_instance("adjoint", seed, m, n,
                           lambda r, k: r.integers(3, 13, k),
                           lambda r, k: r.uniform(1.0, 100.0, k), 1.0)


def paper(seed=5, scale=1.0):
    m = max(32, int(1e7 * scale))
    return random_instance("paper", seed, m, m // 2,
                           lambda r, k: r.integers(5, 16, k),
                           lambda r, k: r.uniform(1.0, 100.0, k), 1.0)


def transit_instance(rng, m_target, T=48, len_lo=2, len_hi=12, n_per_link=5,
                     degrade_fraction=0.10, degrade_lo=0.3, name="transit"):
    """A line network of E segments over T time bins (Section VI's
    time-expanded network, simplified to one line).  Link (e, t) has index
    e*T + t; a trip of L segments from segment e0 departing at bin t0 uses
    links (e0+k, t0+k), k = 0..L-1.  A random `degrade_fraction` of links has
    its capacity scaled by U[degrade_lo, 1] (Section V-D's degradation)."""
    E = max(len_hi, int(round(m_target / T)))
    m = E * T
    n = n_per_link * m
    L = rng.integers(len_lo, len_hi + 1, n)
    L = np.minimum(L, min(E, T))
    e0 = (rng.random(n) * (E - L + 1)).astype(np.int64)
    t0 = (rng.random(n) * (T - L + 1)).astype(np.int64)
    stream = np.repeat(np.arange(n, dtype=np.int64), L)
    starts = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(L, out=starts[1:])
    k = np.arange(stream.size, dtype=np.int64) - starts[stream]
    link = (e0[stream] + k) * T + (t0[stream] + k)
    row_ptr, col_idx = csr_from_pairs(m, n, link, stream)
    c = rng.uniform(1.0, 100.0, m)
    hit = rng.permutation(m)[: int(round(degrade_fraction * m))]
    c[hit] *= rng.uniform(degrade_lo, 1.0, hit.size)
    w = rng.uniform(0.5, 2.0, n)
    utility = np.full(n, LOG, dtype=np.uint8)
    return Instance(name, m, n, row_ptr, col_idx, c, w, utility, 0.0, float(c.max()))


def transit_case_study(seed=8, stations=100, T=192, edges=952, od_pairs=110,
                       routes_per_od=2, departures=90, cap_lo=20.0, cap_hi=60.0):
    """Section VI's time-expanded transit network at its stated size.

    Stations are random points in the unit square.  The spatial network is
    the minimum spanning tree of the complete distance graph plus the shortest
    remaining station pairs until `edges` directed edges (both directions of
    each pair) exist.  A link is an (edge, time bin) pair with index e*T + t;
    every edge takes one bin.  An OD pair gets `routes_per_od` spatial routes:
    the shortest path by length, then shortest paths with the edges already
    used penalised 3x (so the alternatives differ where the network allows).
    A stream j = (OD pair, route, departure t0) with t0 = 0..departures-1
    uses links (e_k, t0 + k) along its route; w_j = 1 log utilities; seat
    capacities U[cap_lo, cap_hi].  The defaults give m = 952 x 192 = 182,784
    links and n = 110 x 2 x 90 = 19,800 streams, the sizes of Section VI's
    case study (whose exact network the paper does not give).

    Returns (Instance, meta) where meta holds per-stream od, route, t0 arrays
    and the spatial routes as lists of edge indices."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra, minimum_spanning_tree

    rng = np.random.default_rng(seed)
    pts = rng.random((stations, 2))
    dist = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1))
    mst = minimum_spanning_tree(csr_matrix(dist)).tocoo()
    pairs = {(min(a, b), max(a, b)) for a, b in zip(mst.row.tolist(), mst.col.tolist())}
    iu, ju = np.triu_indices(stations, 1)
    for k in np.argsort(dist[iu, ju], kind="stable"):
        if len(pairs) * 2 >= edges:
            break
        pairs.add((int(iu[k]), int(ju[k])))
    und = sorted(pairs)
    src = np.array([a for a, b in und] + [b for a, b in und], dtype=np.int64)
    dst = np.array([b for a, b in und] + [a for a, b in und], dtype=np.int64)
    E = src.size
    if E != edges:
        raise ValueError("edge count not reachable")
    eid = {(int(a), int(b)): e for e, (a, b) in enumerate(zip(src, dst))}
    length = dist[src, dst]

    def shortest(o, d, weight):
        g = csr_matrix((weight, (src, dst)), shape=(stations, stations))
        _, pred = dijkstra(g, indices=o, return_predecessors=True)
        path, v = [], d
        while v != o:
            u = int(pred[v])
            path.append(eid[(u, v)])
            v = u
        return path[::-1]

    od = []
    while len(od) < od_pairs:
        o, d = (int(v) for v in rng.choice(stations, 2, replace=False))
        if (o, d) not in od:
            od.append((o, d))
    routes = []
    for o, d in od:
        weight = length.copy()
        rs = []
        for _ in range(routes_per_od):
            r = shortest(o, d, weight)
            rs.append(r)
            weight[r] *= 3.0
        routes.append(rs)
    longest = max(len(r) for rs in routes for r in rs)
    if departures + longest > T:
        raise ValueError("departures do not fit the time horizon")
    links, streams, meta_od, meta_r, meta_t0 = [], [], [], [], []
    j = 0
    for k, rs in enumerate(routes):
        for ri, r in enumerate(rs):
            r_arr = np.asarray(r, dtype=np.int64)
            for t0 in range(departures):
                links.append(r_arr * T + t0 + np.arange(r_arr.size))
                streams.append(np.full(r_arr.size, j, dtype=np.int64))
                meta_od.append(k)
                meta_r.append(ri)
                meta_t0.append(t0)
                j += 1
    m, n = E * T, j
    row_ptr, col_idx = csr_from_pairs(m, n, np.concatenate(links), np.concatenate(streams))
    c = rng.uniform(cap_lo, cap_hi, m)
    inst = Instance("transit_case_study", m, n, row_ptr, col_idx, c, np.ones(n),
                    np.full(n, LOG, dtype=np.uint8), 0.0, float(c.max()))
    meta = {"od": np.asarray(meta_od), "route": np.asarray(meta_r), "t0": np.asarray(meta_t0),
            "routes": routes, "od_pairs": od, "edge_src": src, "edge_dst": dst, "T": T}
    return inst, meta


def batched(seed=3, count=64, m_lo=1e3, m_hi=1e5, scale=1.0):
    """`count` transit instances with m log-uniform on [m_lo, m_hi] (times scale)."""
    rng = np.random.default_rng(seed)
    ms = np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), count)) * scale
    return [transit_instance(rng, max(96.0, float(mt)), name=f"transit{i}")
            for i, mt in enumerate(ms)]


def paper_example(c1=1.0, c=3.0, w=(1.0, 1.0, 1.0, 1.0), hi=math.inf):
    """The 3-link, 4-stream network of Section III-A (all log utilities)."""
    row_ptr = np.array([0, 1, 3, 5], dtype=np.int32)
    col_idx = np.array([0, 1, 2, 1, 3], dtype=np.int32)
    return Instance("paper_example", 3, 4, row_ptr, col_idx,
                    np.array([c1, c, c], dtype=np.float64),
                    np.asarray(w, dtype=np.float64),
                    np.zeros(4, dtype=np.uint8), 0.0, hi)


def single_link(w, utility, cap, lo=0.0, hi=math.inf):
    """All streams share one link."""
    n = len(w)
    return Instance("single_link", 1, n, np.array([0, n], dtype=np.int32),
                    np.arange(n, dtype=np.int32), np.array([cap], dtype=np.float64),
                    np.asarray(w, dtype=np.float64), np.asarray(utility, dtype=np.uint8),
                    lo, hi)


def block_diagonal(parts):
    """Disjoint union of instances (links and streams of each part kept apart)."""
    m = sum(p.m for p in parts)
    n = sum(p.n for p in parts)
    row_ptr = [np.zeros(1, dtype=np.int64)]
    cols, off_nnz, off_n = [], 0, 0
    for p in parts:
        row_ptr.append(p.row_ptr[1:].astype(np.int64) + off_nnz)
        cols.append(p.col_idx.astype(np.int64) + off_n)
        off_nnz += p.nnz
        off_n += p.n
    lo = parts[0].lo
    hi = parts[0].hi
    if any(p.lo != lo or p.hi != hi for p in parts):
        raise ValueError("parts must share the box")
    return Instance("block", m, n, np.concatenate(row_ptr).astype(np.int32),
                    np.concatenate(cols).astype(np.int32),
                    np.concatenate([p.c for p in parts]),
                    np.concatenate([p.w for p in parts]),
                    np.concatenate([p.utility for p in parts]).astype(np.uint8), lo, hi)


def edge_shapes(seed=11, m=6000, n=9000, hi=20.0):
    """Ragged shapes for parity tests: stream 0 on a route of 5000 links
    (longer than one workgroup's 4096-entry stage), the last link on 4500
    streams, links m-10 .. m-2 on no stream, stream n-1 with an empty route
    (its rate is then hi, so hi must be finite), and the rest on routes of
    1-3 links; 30% linear utilities."""
    rng = np.random.default_rng(seed)
    link, stream = [], []
    long_route = rng.choice(m - 10, 5000, replace=False)         # stream 0
    link += list(long_route)
    stream += [0] * 5000
    busy = m - 1                                                  # link on 4500 streams
    for j in range(1, 4501):
        link.append(busy)
        stream.append(j)
    for j in range(1, n - 1):                                     # stream n-1: empty route
        L = int(rng.integers(1, 4))
        for l in rng.choice(m - 10, L, replace=False):
            if not (j <= 4500 and l == busy):
                link.append(int(l))
                stream.append(j)
    pairs = np.unique(np.array([link, stream]).T, axis=0)
    row_ptr, col_idx = csr_from_pairs(m, n, pairs[:, 0], pairs[:, 1])
    util = (rng.random(n) < 0.3).astype(np.uint8)
    w = np.where(util == 0, rng.uniform(0.5, 2, n), rng.uniform(0.1, 1, n))
    return Instance("edge", m, n, row_ptr, col_idx, rng.uniform(1, 50, m), w, util, 0.0, hi)


def congested(base, link_frac=0.001, stream_frac=0.10, seed=6):
    """Section V-C's congestion: a random `link_frac` of the links is each
    added to the routes of a random `stream_frac` of the streams (pairs that
    already exist are kept once).  Capacities and weights are kept."""
    rng = np.random.default_rng(seed)
    m, n = base.m, base.n
    k = max(1, int(round(link_frac * m)))
    hot = rng.choice(m, k, replace=False)
    per = max(1, int(round(stream_frac * n)))
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(base.row_ptr))
    links = [rows, np.repeat(hot.astype(np.int64), per)]
    streams = [base.col_idx.astype(np.int64)]
    for _ in hot:
        streams.append(rng.choice(n, per, replace=False).astype(np.int64))
    key = np.unique(np.concatenate(links) * n + np.concatenate(streams))
    row_ptr, col_idx = csr_from_pairs(m, n, key // n, key % n)
    return Instance(base.name + "_congested", m, n, row_ptr, col_idx, base.c, base.w,
                    base.utility, base.lo, base.hi)


CONFIGS = {"tiny": tiny, "medium": medium, "large": large, "adjoint": adjoint,
           "paper": paper}


def make(name, seed=None, scale=1.0):
    fn = CONFIGS[name]
    return fn(scale=scale) if seed is None else fn(seed=seed, scale=scale)
