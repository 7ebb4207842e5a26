"""Brute-force segmentation used to pin the oracle.

Independent of the oracle on purpose: the edges come from explicitly
enumerated Kuhn simplices (every cube split along the monotone lattice paths
from its low to its high corner, one simplex per permutation of the axes),
"higher" is the plain tuple comparison (value, index) with no order field, and
labels come from walking each integral line to its end.  Pure Python; meant
for grids of a few hundred vertices.
"""
from __future__ import annotations

import itertools

import numpy as np


def kuhn_edges(nx: int, ny: int, nz: int):
    """Adjacency sets of the triangulated grid, built from its top simplices."""
    dims = (nx, ny, nz)
    axes = [a for a in range(3) if dims[a] > 1]
    adj = [set() for _ in range(nx * ny * nz)]

    def vid(p):
        return p[0] + nx * (p[1] + ny * p[2])

    ranges = [range(dims[a] - 1) if a in axes else range(1) for a in range(3)]
    for corner in itertools.product(*ranges):
        for perm in itertools.permutations(axes):
            path = [list(corner)]
            for a in perm:
                p = list(path[-1])
                p[a] += 1
                path.append(p)
            ids = [vid(p) for p in path]
            for i in ids:
                for j in ids:
                    if i != j:
                        adj[i].add(j)
    return adj


def segment(field: np.ndarray):
    """(asc, desc, ms, K) of a field given as an (nz, ny, nx), (ny, nx) or
    (nx,) array."""
    f = np.asarray(field)
    shape = f.shape
    if f.ndim == 1:
        nx, ny, nz = shape[0], 1, 1
    elif f.ndim == 2:
        nx, ny, nz = shape[1], shape[0], 1
    else:
        nx, ny, nz = shape[2], shape[1], shape[0]
    vals = [float(a) for a in f.ravel()]
    n = len(vals)
    adj = kuhn_edges(nx, ny, nz)

    def higher(u, w):
        return (vals[u], u) > (vals[w], w)

    def walk(v, up):
        while True:
            best = v
            for x in adj[v]:
                if (higher(x, best) if up else higher(best, x)):
                    best = x
            if best == v:
                return v
            v = best

    desc = [walk(v, True) for v in range(n)]
    asc = [walk(v, False) for v in range(n)]
    pairs = sorted(set(zip(asc, desc)))
    rank = {p: i for i, p in enumerate(pairs)}
    ms = [rank[p] for p in zip(asc, desc)]
    return (np.array(asc, np.int32).reshape(shape), np.array(desc, np.int32).reshape(shape),
            np.array(ms, np.int32).reshape(shape), len(pairs))


def grid3x3_all_orderings():
    """Labels for every ordering of the values 0..8 on the 3x3 grid, computed
    for all 9! orderings at once.  Returns (perms, asc, desc, ms, K) with perms
    of shape (362880, 9)."""
    adj = kuhn_edges(3, 3, 1)
    perms = np.array(list(itertools.permutations(range(9))), dtype=np.int64)
    m = perms.shape[0]
    vid = np.arange(9)
    up = np.empty((m, 9), np.int64)
    dn = np.empty((m, 9), np.int64)
    for v in range(9):
        cand = np.array(sorted(adj[v] | {v}))
        vals = perms[:, cand]  # values are distinct: no tie-break needed
        up[:, v] = cand[np.argmax(vals, axis=1)]
        dn[:, v] = cand[np.argmin(vals, axis=1)]
    desc, asc = up.copy(), dn.copy()
    for _ in range(9):  # every integral line has at most 8 edges
        desc = np.take_along_axis(desc, desc, axis=1)
        asc = np.take_along_axis(asc, asc, axis=1)
    key = asc * 9 + desc
    present = np.zeros((m, 81), bool)
    present[np.arange(m)[:, None], key] = True
    cum = np.cumsum(present, axis=1)
    ms = np.take_along_axis(cum, key, axis=1) - 1
    k = cum[:, -1]
    del vid
    return perms, asc.astype(np.int32), desc.astype(np.int32), ms.astype(np.int32), k
