"""Pins of the oracle's meshing (Sec. IV, V-B..V-E) against closed forms,
invariants and a brute-force dense marching-cubes check.

- a closed sphere: edge-manifold, oriented outward, Euler characteristic 2,
  V = F/2 + 2, enclosed volume close to 4/3 pi r^3, every vertex within the
  linear-interpolation error bound of the true surface;
- the single-sphere workload literally (r = 0.30 m in a 0.512 m lattice): a
  sphere with six caps cut off -> chi = -4 and six boundary loops;
- a regular plane patch: 2wh triangles on (w+1)(h+1) vertices (Sec. VI-B);
- a linear field: every vertex on the plane;
- exactly one vertex per sign-changing edge of a valid cube (dense brute
  force), reference count = triangle degree (Sec. V-E);
- incremental extraction over a fused sequence equals extraction from
  scratch of the final volume.
"""
import math
import os

import numpy as np
import pytest

import oracle
import scenes
from tests import meshutil

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def mesh_of(vol):
    verts, tris = vol.download()
    return verts, tris


def import_dense(vol, tsdf, w=None):
    coords, d = scenes.dense_to_blocks(tsdf.astype(np.float32))
    if w is None:
        w = np.ones_like(d)
    else:
        _, w = scenes.dense_to_blocks(w.astype(np.float32))
    vol.import_blocks(coords, d, w)


def test_closed_sphere_topology_and_geometry():
    sv = scenes.sphere_volume(seed=1, radius=0.20)
    vol = oracle.OracleVolume(sv.voxel_m)
    import_dense(vol, sv.tsdf)
    vol.extract(scope_all=True)
    verts, tris = mesh_of(vol)
    V, F = len(verts), len(tris)
    good, boundary, bad = meshutil.manifold_report(tris)
    assert bad == 0 and boundary == 0
    assert meshutil.euler_characteristic(V, tris) == 2
    assert V == F // 2 + 2 and F % 2 == 0
    r = sv.meta["radius"]
    vol_enc = meshutil.signed_volume(verts, tris)
    assert vol_enc > 0  # normals point to the outside (d > 0) region
    assert abs(vol_enc / (4 / 3 * math.pi * r ** 3) - 1) < 0.01
    # radial error of a linearly interpolated root of a sphere's distance
    # field: |f(x)| <= max|f''|/8 with |f''| <= 1/(R-1.5) voxels near it
    s = sv.voxel_m
    R = r / s
    err = np.abs(np.linalg.norm(verts.astype(np.float64) - sv.meta["center"], axis=1) - r) / s
    assert err.max() <= 1.0 / (8 * (R - 1.5)) + 1e-4
    # reference counts are vertex degrees, they sum to 3F (Sec. V-E)
    vv = vol.vertices()
    assert vv["ref"].sum() == 3 * F
    assert (np.bincount(tris.ravel(), minlength=V) == vv["ref"]).all()


def test_single_sphere_workload_is_a_capped_sphere():
    sv = scenes.sphere_volume(seed=1)  # r = 0.30 m in the 0.512 m lattice
    vol = oracle.OracleVolume(sv.voxel_m)
    import_dense(vol, sv.tsdf)
    vol.extract(scope_all=True)
    verts, tris = mesh_of(vol)
    good, boundary, bad = meshutil.manifold_report(tris)
    assert bad == 0
    assert meshutil.euler_characteristic(len(verts), tris) == -4
    assert meshutil.boundary_loops(tris) == 6
    # every open edge lies on one of the lattice's outer faces (0 or 63 voxels)
    s = sv.voxel_m
    from collections import Counter
    de = meshutil.directed_edges(tris)
    for (u, v) in de:
        if (v, u) in de:
            continue
        pu, pv = verts[u] / s, verts[v] / s
        on = [a for a in range(3) for b in (0.0, 63.0)
              if abs(pu[a] - b) < 1e-3 and abs(pv[a] - b) < 1e-3]
        assert on


def read_patches():
    rows = []
    for l in open(os.path.join(GOLDEN, "plane_patch.txt")):
        if l.strip() and not l.startswith("#"):
            rows.append(tuple(int(x) for x in l.split()))
    return rows


@pytest.mark.parametrize("w,h,F,V", read_patches())
def test_regular_plane_patch_counts(w, h, F, V):
    # d = z - 7.3 voxels: one layer of cubes crosses it; only voxels with
    # x <= w and y <= h carry weight, so exactly a w x h cube patch is valid.
    Z = Y = X = 16
    g = np.arange(16, dtype=np.float64)
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    tsdf = (zz - 7.3).astype(np.float32)
    wt = ((xx <= w) & (yy <= h)).astype(np.float32)
    vol = oracle.OracleVolume(0.01)
    import_dense(vol, tsdf, wt)
    vol.extract(scope_all=True)
    verts, tris = mesh_of(vol)
    assert (len(tris), len(verts)) == (F, V)
    assert F == 2 * w * h and V == (w + 1) * (h + 1)


def test_linear_field_vertices_lie_on_the_plane():
    rng = np.random.default_rng(7)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    p0 = np.array([7.7, 8.1, 8.3])
    g = np.arange(16, dtype=np.float64)
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    d = n[0] * (xx - p0[0]) + n[1] * (yy - p0[1]) + n[2] * (zz - p0[2])
    vol = oracle.OracleVolume(1.0)
    import_dense(vol, d.astype(np.float32))
    vol.extract(scope_all=True)
    vv = vol.vertices()
    keys, t = vv["keys"], vv["t"].astype(np.float64)
    pos = keys[:, :3].astype(np.float64)
    pos[np.arange(len(t)), keys[:, 3]] += t
    dist = (pos - p0) @ n
    assert len(t) > 100
    assert np.abs(dist).max() < 1e-5
    assert ((t >= 0) & (t <= 1)).all()


def brute_force_vertices(tsdf, w):
    """All edges of valid cubes whose end signs differ, on a dense (Z,Y,X)
    grid, with their FP32 interpolation parameter."""
    Z, Y, X = tsdf.shape
    valid_c = np.zeros((Z - 1, Y - 1, X - 1), bool)
    ok = w > 0
    valid_c = (ok[:-1, :-1, :-1] & ok[:-1, :-1, 1:] & ok[:-1, 1:, :-1] & ok[:-1, 1:, 1:] &
               ok[1:, :-1, :-1] & ok[1:, :-1, 1:] & ok[1:, 1:, :-1] & ok[1:, 1:, 1:])
    out = {}
    neg = tsdf < 0
    for axis, (dz, dy, dx) in enumerate([(0, 0, 1), (0, 1, 0), (1, 0, 0)]):
        for z in range(Z - dz):
            for y in range(Y - dy):
                for x in range(X - dx):
                    if neg[z, y, x] == neg[z + dz, y + dy, x + dx]:
                        continue
                    # cubes containing this edge: anchors differ by 0/-1 in the
                    # two other axes
                    used = False
                    others = [a for a in range(3) if a != axis]
                    for o1 in (0, -1):
                        for o2 in (0, -1):
                            c = [x, y, z]
                            c[others[0]] += o1
                            c[others[1]] += o2
                            cx, cy, cz = c
                            if 0 <= cx < X - 1 and 0 <= cy < Y - 1 and 0 <= cz < Z - 1:
                                used |= bool(valid_c[cz, cy, cx])
                    if used:
                        da = np.float32(tsdf[z, y, x])
                        db = np.float32(tsdf[z + dz, y + dy, x + dx])
                        out[(x, y, z, axis)] = np.float32(da / (da - db))
    return out


@pytest.mark.parametrize("seed", [3, 4])
def test_one_vertex_per_sign_changing_edge_brute_force(seed):
    rng = np.random.default_rng(seed)
    tsdf = rng.uniform(-1.5, 1.5, (16, 16, 16)).astype(np.float32)
    w = (rng.uniform(size=(16, 16, 16)) > 0.1).astype(np.float32)
    vol = oracle.OracleVolume(0.01)
    import_dense(vol, tsdf, w)
    vol.extract(scope_all=True)
    vv = vol.vertices()
    got = {tuple(k): t for k, t in zip(vv["keys"].tolist(), vv["t"])}
    want = brute_force_vertices(tsdf, w)
    assert set(got) == set(want)
    for k, t in want.items():
        assert got[k] == t


def incremental_vs_scratch(seq, frames, refine=False):
    vol = oracle.OracleVolume(seq.voxel_m)
    for k in frames:
        vol.integrate(seq.frame(k), scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        vol.extract()
        if refine:
            vol.refine()
        vol.gc()
    b = vol.blocks()
    fresh = oracle.OracleVolume(seq.voxel_m)
    fresh.import_blocks(b["coords"], b["d"], b["w"])
    fresh.extract(scope_all=True)
    fresh.gc()
    return vol, fresh


def test_incremental_equals_from_scratch():
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.04)
    vol, fresh = incremental_vs_scratch(seq, [0, 7, 14])
    a, b = vol.vertices(live_only=False), fresh.vertices(live_only=False)
    assert len(a["keys"]) > 1000
    assert (a["keys"] == b["keys"]).all()
    assert (a["t"] == b["t"]).all()
    assert (a["ref"] == b["ref"]).all() and (a["ref"] > 0).all()
    assert (meshutil.canonical_triangles(vol.triangles()) ==
            meshutil.canonical_triangles(fresh.triangles())).all()
    assert (vol.blocks()["cur"] == fresh.blocks()["cur"]).all()


def test_gc_frees_exactly_the_unreferenced_vertices():
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.04)
    vol = oracle.OracleVolume(seq.voxel_m)
    for k in (0, 5):
        vol.integrate(seq.frame(k), scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        vol.extract()
    allv = vol.vertices(live_only=False)
    dead = int((allv["ref"] == 0).sum())
    assert dead > 0  # the second frame moved some surface
    assert (allv["ref"] >= 0).all()
    assert vol.gc() == dead
    after = vol.vertices(live_only=False)
    assert (after["ref"] > 0).all()
    # every remaining vertex is used by a triangle and vice versa
    used = {tuple(k) for tri in vol.triangles().tolist() for k in tri}
    assert used == {tuple(k) for k in after["keys"].tolist()}


def test_an_edge_can_carry_more_than_fifteen_triangles():
    """Reference counts need more than four bits: the four cubes around an
    edge can each use it in four triangles (brute force over all 2^18 sign
    patterns of their corners).  A crossing edge is used by every one of the
    four cubes, so a count is 0 or at least 4."""
    from tests.edge_load import edge_loads
    load, pats = edge_loads()
    assert load.max() == 16
    counts = set(np.unique(load).tolist())
    assert counts == {0} | set(range(4, 17))
