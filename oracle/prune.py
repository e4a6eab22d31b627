"""Link failure and pruning of a NUM instance -- test infrastructure.

Only the tests and the benchmark's CPU-baseline leg use this module; the HIP
library never imports or calls it.

Section V-D re-solves after links fail.  Reading used here: a failed link
leaves the network together with every stream whose route crosses it (that
path is broken and the stream is not rerouted); every other link and stream
stays, numbered in its old order, and the warm start is the previous iterate
restricted to the survivors.  Written as the plain definition: the surviving
sets, then the submatrix R[keep_links, keep_streams].
"""
from __future__ import annotations

import numpy as np


def survivors(inst, failed):
    """Boolean masks (links kept [m], streams kept [n]) for failed[m] != 0."""
    failed = np.asarray(failed).astype(bool)
    rows = np.repeat(np.arange(inst.m), np.diff(inst.row_ptr))
    dead = np.zeros(inst.n, bool)
    dead[inst.col_idx[failed[rows]]] = True
    return ~failed, ~dead


def prune(inst, failed):
    """Pruned CSR and vectors.

    Returns a dict with m, n, nnz, row_ptr, col_idx (int32), c, w, utility,
    link_map (old index of each kept link), stream_map (old index of each
    kept stream)."""
    keep_l, keep_s = survivors(inst, failed)
    link_map = np.flatnonzero(keep_l).astype(np.int32)
    stream_map = np.flatnonzero(keep_s).astype(np.int32)
    new_s = np.full(inst.n, -1, np.int64)
    new_s[stream_map] = np.arange(stream_map.size)
    row_ptr = [0]
    cols = []
    for l in link_map:
        seg = inst.col_idx[inst.row_ptr[l]:inst.row_ptr[l + 1]]
        kept = new_s[seg[keep_s[seg]]]
        cols.append(kept)
        row_ptr.append(row_ptr[-1] + kept.size)
    col_idx = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    return {"m": int(link_map.size), "n": int(stream_map.size), "nnz": int(col_idx.size),
            "row_ptr": np.asarray(row_ptr, np.int32), "col_idx": col_idx,
            "c": np.asarray(inst.c)[link_map], "w": np.asarray(inst.w)[stream_map],
            "utility": np.asarray(inst.utility)[stream_map],
            "link_map": link_map, "stream_map": stream_map}


def restrict_state(a, b, zs, u, link_map, stream_map):
    """The warm start: the iterate restricted to the survivors."""
    return a[stream_map], b[link_map], zs[link_map], u[link_map]
