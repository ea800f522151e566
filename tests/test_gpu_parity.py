"""GPU library vs CPU oracle, through the C-ABI, on seeded synthetic inputs.

Bar: hash membership, cube types, vertex set, reference counts and triangle
connectivity bit-exact; TSDF, weights and edge parameters within 1e-5 voxel
units (in practice they are bit-identical: both sides run the same FP32
operations without contraction and with correctly rounded division)."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from tests import meshutil
from tests.gpu_compare import compare_all, compare_blocks, compare_triangles, compare_vertices, to_dev

pytestmark = pytest.mark.gpu


def new_volume(voxel_m, **kw):
    from paper_1803_03949_amd import Volume
    args = dict(hash_log2=16, max_blocks=1 << 14, max_vertices=1 << 20)
    args.update(kw)
    return Volume(voxel_m, **args)


def import_both(sv_or_blocks, voxel_m, gkw=None, eps=0.5):
    if hasattr(sv_or_blocks, "blocks"):
        coords, d, w = sv_or_blocks.blocks()
    else:
        coords, d, w = sv_or_blocks
    g = new_volume(voxel_m, refine_eps_vox=eps, **(gkw or {}))
    g.import_blocks(*to_dev(coords, d, w))
    o = oracle.OracleVolume(voxel_m, 4.0, eps)
    o.import_blocks(coords, d, w)
    return g, o


@pytest.mark.parametrize("radius", [0.30, 0.20])
def test_sphere_extraction(radius):
    print(f"[parity] sphere r={radius}", flush=True)
    sv = scenes.sphere_volume(seed=1, radius=radius)
    g, o = import_both(sv, sv.voxel_m)
    g.extract(scope_all=True)
    o.extract(scope_all=True)
    info = compare_all(g, o)
    assert info["nv"] > 5000
    g.gc()
    o.gc()
    compare_all(g, o)
    st = g.status()
    assert st["error"] == 0 and st["blocks"] == 512


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_sign_fields_cover_all_cube_types(seed):
    print(f"[parity] random field seed={seed}", flush=True)
    rng = np.random.default_rng(seed)
    d = (rng.choice([-1.0, 1.0], size=(16, 16, 16)) * rng.uniform(0.05, 1.0, (16, 16, 16)))
    w = (rng.uniform(size=(16, 16, 16)) > 0.03).astype(np.float32)
    coords, db = scenes.dense_to_blocks(d.astype(np.float32))
    _, wb = scenes.dense_to_blocks(w)
    g, o = import_both((coords, db, wb), 0.01)
    g.extract(scope_all=True)
    o.extract(scope_all=True)
    compare_all(g, o)
    cur = o.blocks()["cur"]
    assert len(np.unique(cur)) == 256


def test_dirty_extraction_after_import_equals_all():
    sv = scenes.sphere_volume(seed=3, dims_blocks=(4, 4, 4), radius=0.14, center=np.full(3, 0.128))
    g, o = import_both(sv, sv.voxel_m)
    g.extract(scope_all=False)
    o.extract(scope_all=False)
    compare_all(g, o)
    assert len(g.block_list("dirty")) == 64


def run_sequence(seq, frames, gkw, refine=False, check_every=True):
    """refine: False, True (a refinement pass after each extraction) or
    "fused" (extraction with the refinement applied to each new type)."""
    g = new_volume(seq.voxel_m, **gkw)
    o = oracle.OracleVolume(seq.voxel_m, 4.0, 0.5)
    for k in frames:
        print(f"[parity] frame {k}", flush=True)
        depth = seq.frame(k)
        g.integrate(to_dev(depth)[0], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        o.integrate(depth, scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        gf = {tuple(x) for x in g.block_list("frame").tolist()}
        of = {tuple(x) for x in o.block_set("frame").tolist()}
        assert gf == of, "collected blocks differ"
        if check_every:
            compare_blocks(g, o, types=False)
        g.extract(refine=refine == "fused")
        o.extract(refine=refine == "fused")
        gd = {tuple(x) for x in g.block_list("dirty").tolist()}
        od = {tuple(x) for x in o.block_set("dirty").tolist()}
        assert gd == od, "dirty blocks differ"
        if refine is True:
            g.refine()
            o.refine()
        if check_every:
            compare_all(g, o)
        g.gc()
        o.gc()
        if check_every:
            compare_vertices(g, o)
    return g, o


def test_room_sequence_coarse():
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.03)
    g, o = run_sequence(seq, [0, 3, 9, 27], dict(hash_log2=16, max_blocks=1 << 14))
    info = compare_all(g, o)
    assert info["nv"] > 10000
    assert g.status()["error"] == 0


def test_room_sequence_8mm_two_frames():
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.008)
    g, o = run_sequence(seq, [0, 1], dict(hash_log2=20, max_blocks=1 << 16, max_vertices=1 << 22), check_every=False)
    info = compare_all(g, o)
    assert info["nv"] > 100000


def test_room_sequence_with_holes_and_refinement():
    seq = scenes.room_sequence(seed=3, n_frames=500, voxel_m=0.03, holes=True)
    g, o = run_sequence(seq, [0, 4, 8, 12], dict(hash_log2=16, max_blocks=1 << 14), refine=True)
    compare_all(g, o)
    assert g.status()["refined_cubes"] >= 0


def test_room_sequence_with_holes_and_refining_extraction():
    seq = scenes.room_sequence(seed=3, n_frames=500, voxel_m=0.03, holes=True)
    g, o = run_sequence(seq, [0, 4, 8, 12, 16], dict(hash_log2=16, max_blocks=1 << 14), refine="fused")
    info = compare_all(g, o)
    assert info["nv"] > 5000 and g.status()["error"] == 0


def test_refining_extraction_counts_and_later_refinement_pass():
    """The refined-cube count of a refining extraction equals the cubes the
    oracle's separate refinement pass re-types; a refinement pass after it
    changes nothing on either side (Eqs. 3-5 are idempotent)."""
    seq = scenes.room_sequence(seed=5, n_frames=500, voxel_m=0.02, holes=True)
    g = new_volume(seq.voxel_m)
    o = oracle.OracleVolume(seq.voxel_m, 4.0, 0.5)
    o2 = oracle.OracleVolume(seq.voxel_m, 4.0, 0.5)
    total = 0
    for k in (0, 3, 6):
        print(f"[parity] refining extraction frame {k}", flush=True)
        depth = seq.frame(k)
        g.integrate(to_dev(depth)[0], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        for ov in (o, o2):
            ov.integrate(depth, scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        g.extract(refine=True)
        o.extract(refine=True)
        o2.extract()
        n_ref = o2.refine()
        assert g.status()["refined_cubes"] == n_ref
        total += n_ref
        g.refine()
        assert o.refine() == 0
        assert g.status()["refined_cubes"] == 0
        compare_all(g, o)
        g.gc()
        o.gc()
        o2.gc()
    assert total > 0


def test_collide_hash_mode_gives_same_volume():
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.06)
    g, o = run_sequence(seq, [0, 5], dict(hash_log2=12, max_blocks=2048, hash_mode=1))
    compare_all(g, o)


def test_incremental_equals_from_scratch_on_gpu():
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.03)
    g = new_volume(seq.voxel_m)
    for k in (0, 6, 12):
        g.integrate(to_dev(seq.frame(k))[0], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        g.extract()
        g.gc()
    b = g.export_blocks()
    f = new_volume(seq.voxel_m)
    f.import_blocks(to_dev(b["coords"])[0], b["d"].contiguous(), b["w"].contiguous())
    f.extract(scope_all=True)
    f.gc()
    from tests.gpu_compare import gpu_live_vertices, gpu_triangle_keys
    a, c = gpu_live_vertices(g), gpu_live_vertices(f)
    assert (a[0] == c[0]).all() and (a[1] == c[1]).all() and (a[2] == c[2]).all()
    ta = meshutil.canonical_triangles(gpu_triangle_keys(g)[0])
    tb = meshutil.canonical_triangles(gpu_triangle_keys(f)[0])
    assert (ta == tb).all()


def test_mesh_is_closed_and_oriented_on_gpu():
    sv = scenes.sphere_volume(seed=1, radius=0.20)
    g, _ = import_both(sv, sv.voxel_m)
    g.extract(scope_all=True)
    g.gc()
    verts, tris, _ = g.download()
    v, t = verts.cpu().numpy(), tris.cpu().numpy()
    good, boundary, bad = meshutil.manifold_report(t)
    assert boundary == 0 and bad == 0
    assert meshutil.euler_characteristic(len(v), t) == 2
    assert meshutil.signed_volume(v, t) > 0


@pytest.mark.parametrize("which", ["blocks", "vertices", "hash"])
def test_capacity_errors_are_reported(which):
    from paper_1803_03949_amd import VmError
    sv = scenes.sphere_volume(seed=1, dims_blocks=(4, 4, 4), radius=0.12, center=np.full(3, 0.128))
    kw = dict(hash_log2=16, max_blocks=1 << 10, max_vertices=1 << 16)
    if which == "blocks":
        kw["max_blocks"] = 40
    elif which == "vertices":
        kw["max_vertices"] = 100
    else:
        kw["hash_log2"] = 10  # 1024 slots, but the integration below collects more blocks
    g = new_volume(sv.voxel_m, **kw)
    coords, d, w = sv.blocks()
    if which == "hash":
        seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.008)
        g.integrate(to_dev(seq.frame(0))[0], scenes.K, seq.poses[0], 0.4, 3.0)
    elif which == "blocks":
        # two imports of 32 blocks: the second one runs out of pool
        g.import_blocks(*to_dev(coords[:32], d[:32], w[:32]))
        g.import_blocks(*to_dev(coords[32:], d[32:], w[32:]))
        g.extract(scope_all=True)
    else:
        g.import_blocks(*to_dev(coords, d, w))
        g.extract(scope_all=True)
    st = g.status(check=False)
    want = {"blocks": -3, "vertices": -4, "hash": -2}[which]
    assert st["error"] == want, st
    with pytest.raises(VmError):
        g.status()


@pytest.mark.parametrize("origin", [(3, 3, 3), (7, 8, 8), (7, 7, 7), (8, 8, 8)])
def test_most_loaded_edges(origin):
    """Edges carrying 16 triangles (the most any edge can), inside a block
    and across block faces, edges and corners: counts, vertices and
    triangles as the oracle's."""
    from tests.edge_load import POINTS, edge_loads
    load, pats = edge_loads()
    best = pats[load == load.max()]
    tsdf = np.full((16, 16, 16), 2.0, np.float32)  # (z, y, x)
    for j, pat in enumerate(best[:3]):
        gx, gy, gz = origin[0], origin[1], origin[2]
        shift = 0 if j == 0 else (j * 5) % 6
        for i, (x, y, z) in enumerate(POINTS):
            inside = (int(pat) >> i) & 1
            tsdf[gz + z, gy + y, (gx + x + shift) % 16] = -0.5 if inside else 0.5
    dense = scenes.DenseVolume(0.01, (2, 2, 2), tsdf, np.ones_like(tsdf))
    g, o = import_both(dense, 0.01)
    g.extract(scope_all=True)
    o.extract(scope_all=True)
    compare_all(g, o)
    assert int(o.vertices()["ref"].max()) == 16


def test_wide_truncation_band():
    """A truncation band several blocks deep: pixel boxes of up to 5^3
    blocks (beyond the per-lane batch of the collection kernel)."""
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.03)
    g = new_volume(seq.voxel_m, trunc_vox=14.0)
    o = oracle.OracleVolume(seq.voxel_m, 14.0, 0.5)
    for k in (0, 7):
        depth = seq.frame(k)
        g.integrate(to_dev(depth)[0], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        o.integrate(depth, scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        gf = {tuple(x) for x in g.block_list("frame").tolist()}
        of = {tuple(x) for x in o.block_set("frame").tolist()}
        assert gf == of
        g.extract()
        o.extract()
    compare_all(g, o)


def test_mesh_size_counters_match_oracle():
    """The counters the mesh-memory report reads (status triangles, live
    vertex slots, blocks) against the oracle's mesh after every frame: the
    report's V and F are these numbers (Sec. VI-B compares vertex counts)."""
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.03)
    g = new_volume(seq.voxel_m)
    o = oracle.OracleVolume(seq.voxel_m, 4.0, 0.5)
    for k in range(0, 30, 3):
        depth = seq.frame(k)
        g.integrate(to_dev(depth)[0], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        o.integrate(depth, scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        g.extract()
        o.extract()
        g.gc()
        o.gc()
        st = g.status()
        nv = len(o.vertices()["keys"])
        nt = len(o.triangles())
        assert st["vertex_slots"] - st["free_vertex_slots"] == nv, k
        assert st["triangles"] == nt, k
        assert st["blocks"] == len(o.blocks()["coords"]), k
        # a vertex count above half the triangle count is what a shared-vertex
        # mesh must show (Sec. VI-B); a soup would hold 3F
        assert nt / 2 <= nv < 3 * nt, k
