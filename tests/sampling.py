"""Sampled parity at full size: the state of a full run compared with the
oracle restricted to the 3x3x3 neighbourhoods of a few sampled blocks.

Collection and fusion of a block depend only on the depth frames and on the
block itself; the mesh inside a block (cube types and their history, the
vertices it owns with their counts, the triangles of its cubes) depends only
on the blocks of its neighbourhood.  The oracle restricted to those
neighbourhoods therefore reproduces the sampled blocks exactly."""
from __future__ import annotations

import numpy as np

from tests import meshutil

TOL = 1e-5  # voxel units


def neighbourhood(coords):
    out = set()
    for c in coords:
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    out.add((c[0] + dx, c[1] + dy, c[2] + dz))
    return np.array(sorted(out), np.int32)


def state(blocks, vkeys, vt, vref, tri_keys):
    """(blocks dict of numpy arrays, coord -> row, edge -> (t, count) of live
    vertices, (F, 3, 4) triangle edge keys)."""
    rows = {tuple(c): i for i, c in enumerate(blocks["coords"].tolist())}
    verts = {tuple(k): (t, r) for k, t, r in zip(vkeys.tolist(), vt, vref) if r > 0}
    return blocks, rows, verts, np.asarray(tri_keys).reshape(-1, 3, 4)


def oracle_state(o):
    b = o.blocks()
    v = o.vertices()
    return state(b, v["keys"], v["t"], v["ref"], o.triangles())


def owner_block(e):
    return (e[0] // 8, e[1] // 8, e[2] // 8)


def triangle_blocks(tris):
    """For each triangle ((F, 3, 4) edge keys), the block of the smallest
    owner coordinate along each axis.  A triangle's edges are owned by
    corners of its cube, so along an axis the cube's minimum corner is that
    smallest coordinate, or one less when all three owners share it (a
    triangle lying in a cube face).  A triangle whose smallest-owner block is
    s therefore belongs to a cube of s or of one of its -x/-y/-z neighbours,
    whose histories the restricted oracle reproduces exactly; and every
    triangle of a cube of s is among them."""
    lo = np.asarray(tris)[:, :, :3].min(axis=1)
    return np.floor_divide(lo, 8)


def triangles_of_block(tris, blocks_of, s):
    sel = np.asarray(tris)[(blocks_of == np.array(s)).all(axis=1)]
    return meshutil.canonical_triangles(sel.reshape(-1, 3, 4))


def check_samples(full, o, samples):
    """Compare a full run's state with the restricted oracle `o` on the
    sampled blocks."""
    b, blocks, verts, ek = full
    ob, orow, overts, otri = oracle_state(o)
    ek_blocks, otri_blocks = triangle_blocks(ek), triangle_blocks(otri)
    wanted = set(map(tuple, samples.tolist()))
    by_owner_g, by_owner_o = {}, {}
    for src, dst in ((verts, by_owner_g), (overts, by_owner_o)):
        for k, v in src.items():
            ob_k = owner_block(k)
            if ob_k in wanted:
                dst.setdefault(ob_k, {})[k] = v
    for s in map(tuple, samples.tolist()):
        # membership of the whole neighbourhood
        for n in map(tuple, neighbourhood([s]).tolist()):
            assert (n in blocks) == (n in orow), n
        if s not in blocks:
            continue
        i, j = blocks[s], orow[s]
        d = np.asarray(b["d"][i], np.float64)
        w = np.asarray(b["w"][i], np.float64)
        assert np.abs(d - ob["d"][j]).max() <= TOL and np.abs(w - ob["w"][j]).max() <= TOL, s
        assert np.array_equal(b["cur"][i], ob["cur"][j]), s
        assert np.array_equal(b["prev"][i], ob["prev"][j]), s
        # vertices the block owns
        mine_g = by_owner_g.get(s, {})
        mine_o = by_owner_o.get(s, {})
        assert mine_g.keys() == mine_o.keys(), s
        for k in mine_g:
            assert mine_g[k][1] == mine_o[k][1], (s, k)
            assert abs(float(mine_g[k][0]) - float(mine_o[k][0])) <= TOL, (s, k)
        # triangles of the block's cubes
        tg = triangles_of_block(ek, ek_blocks, s)
        to = triangles_of_block(otri, otri_blocks, s)
        assert tg.shape == to.shape and (tg == to).all(), s


def check_invariants(full):
    """Properties of any mesh the method produces: the reference count of
    every live vertex is the number of triangles using it, and every edge a
    triangle uses holds a live vertex."""
    b, blocks, verts, ek = full
    counts = {}
    for tri in ek.tolist():
        for e in tri:
            counts[tuple(e)] = counts.get(tuple(e), 0) + 1
    assert counts.keys() == verts.keys()
    assert all(verts[k][1] == c for k, c in counts.items())
    assert sum(r for _, r in verts.values()) == 3 * len(ek)


def sample_blocks(blocks, rng, n_in, n_out):
    have = list(blocks.keys())
    picks = [have[i] for i in rng.choice(len(have), n_in, replace=False)]
    out = []
    for i in rng.permutation(len(have)):
        c = have[i]
        n = (c[0] + 2, c[1], c[2] - 2)
        if n not in blocks:
            out.append(n)
        if len(out) == n_out:
            break
    return np.array(picks + out, np.int32)


