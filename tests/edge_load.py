"""Sign patterns around one lattice edge that load it with the most
triangles: a brute force over the 18 lattice points of the four cubes that
share an x-edge, counting with the oracle's own triangle lists."""
from __future__ import annotations

import numpy as np

import oracle


def uses_table() -> np.ndarray:
    """uses[t, e]: triangles of cube type t that use cube edge e."""
    u = np.zeros((256, 12), np.int64)
    for t in range(256):
        for tri in oracle.cube_triangles(t):
            for e in tri:
                u[t, e] += 1
    return u


# The four cubes around the x-edge from (0,0,0) to (1,0,0): anchors at
# (0, -dy, -dz); for each, the cube edge the shared edge is (e0, e2, e4, e6).
CUBES = [((0, 0, 0), 0), ((0, -1, 0), 2), ((0, 0, -1), 4), ((0, -1, -1), 6)]
POINTS = [(x, y, z) for z in (-1, 0, 1) for y in (-1, 0, 1) for x in (0, 1)]


def edge_loads() -> tuple[np.ndarray, np.ndarray]:
    """(loads, patterns): for every sign pattern (bit i set: POINTS[i] is
    inside), the number of triangles using the shared edge."""
    corners = oracle.corner_offsets()
    u = uses_table()
    pats = np.arange(1 << len(POINTS), dtype=np.int64)
    index = {p: i for i, p in enumerate(POINTS)}
    load = np.zeros(len(pats), np.int64)
    for anchor, edge in CUBES:
        t = np.zeros(len(pats), np.int64)
        for k, off in enumerate(corners.tolist()):
            p = (anchor[0] + off[0], anchor[1] + off[1], anchor[2] + off[2])
            t |= ((pats >> index[p]) & 1) << k
        load += u[t, edge]
    return load, pats
