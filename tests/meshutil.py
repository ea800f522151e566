"""Mesh topology and comparison helpers for the tests (not part of the method)."""
from __future__ import annotations

from collections import Counter

import numpy as np


def undirected_edges(tris: np.ndarray) -> Counter:
    c = Counter()
    for a, b, d in np.asarray(tris):
        for u, v in ((a, b), (b, d), (d, a)):
            c[(min(u, v), max(u, v))] += 1
    return c


def directed_edges(tris: np.ndarray) -> Counter:
    c = Counter()
    for a, b, d in np.asarray(tris):
        for u, v in ((a, b), (b, d), (d, a)):
            c[(int(u), int(v))] += 1
    return c


def manifold_report(tris: np.ndarray):
    """Counts of (interior edges used twice with opposite orientation,
    boundary edges used once, bad edges)."""
    de = directed_edges(tris)
    ue = undirected_edges(tris)
    good = boundary = bad = 0
    for (u, v), n in ue.items():
        if n == 2 and de.get((u, v), 0) == 1 and de.get((v, u), 0) == 1:
            good += 1
        elif n == 1:
            boundary += 1
        else:
            bad += 1
    return good, boundary, bad


def euler_characteristic(nverts: int, tris: np.ndarray) -> int:
    return nverts - len(undirected_edges(tris)) + len(tris)


def boundary_loops(tris: np.ndarray) -> int:
    de = directed_edges(tris)
    bnd = [(u, v) for (u, v) in de if (v, u) not in de]
    nxt = {}
    for u, v in bnd:
        nxt.setdefault(u, []).append(v)
    seen = set()
    loops = 0
    for u, v in bnd:
        if (u, v) in seen:
            continue
        loops += 1
        cur = (u, v)
        while cur not in seen:
            seen.add(cur)
            cands = [w for w in nxt.get(cur[1], []) if (cur[1], w) not in seen]
            if not cands:
                break
            cur = (cur[1], cands[0])
    return loops


def signed_volume(verts: np.ndarray, tris: np.ndarray) -> float:
    v = np.asarray(verts, np.float64)
    t = np.asarray(tris)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def canonical_triangles(keys: np.ndarray) -> np.ndarray:
    """Triangles given as (F, 3, K) integer keys -> (F, 3K) rows, each rotated
    so its smallest key comes first (orientation kept), rows sorted."""
    keys = np.asarray(keys)
    F = keys.shape[0]
    if F == 0:
        return keys.reshape(0, 3 * keys.shape[2] if keys.ndim == 3 else 0)
    flat = [tuple(map(tuple, tri)) for tri in keys]
    out = []
    for tri in flat:
        i = min(range(3), key=lambda j: tri[j])
        rot = tri[i:] + tri[:i]
        out.append(sum(rot, ()))
    out.sort()
    return np.array(out, dtype=np.int64)


def sort_rows(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a)
    if len(a) == 0:
        return a
    idx = np.lexsort(a.T[::-1])
    return a[idx]
