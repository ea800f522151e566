"""Vertex pool segments: the block at pool row b creates its vertices in
segment b mod n only, each segment holding ceil(max_vertices / n) slots.
A surface crowded into the blocks of one segment therefore fills that
segment before the pool: the error is raised exactly when the fullest
segment's share is exceeded, the status reports the segment layout and the
fullest segment, and a pool fitted to that segment meshes as the oracle
does."""
import numpy as np
import pytest

import oracle
import scenes
from paper_1803_03949_amd import Volume
from tests.gpu_compare import compare_all, to_dev

pytestmark = pytest.mark.gpu

NSEG = 4          # max_blocks 1024: one segment per 256 blocks of capacity
MAX_BLOCKS = 1024


def skewed_blocks():
    """A sphere's 64 blocks on pool rows 0, 4, 8, ... (all in segment 0) and
    far-away empty blocks (TSDF +4, no surface) on the rows between."""
    sv = scenes.sphere_volume(seed=3, dims_blocks=(4, 4, 4), voxel_m=0.01, radius=0.11,
                              center=np.full(3, 0.16), jitter=0.005)
    c, d, w = sv.blocks()
    n = len(c)
    coords = np.zeros((NSEG * n, 3), np.int32)
    tsdf = np.full((NSEG * n, 512), 4.0, np.float32)
    weight = np.ones((NSEG * n, 512), np.float32)
    coords[0::NSEG] = c
    tsdf[0::NSEG] = d
    weight[0::NSEG] = w
    filler = np.arange(n * (NSEG - 1))
    rest = np.flatnonzero(np.arange(NSEG * n) % NSEG)
    coords[rest] = np.stack([100 + 2 * (filler % 20), 100 + 2 * (filler // 20),
                             np.full_like(filler, 100)], 1)
    return sv, coords, tsdf, weight


def run(max_vertices):
    sv, coords, tsdf, weight = skewed_blocks()
    g = Volume(sv.voxel_m, hash_log2=12, max_blocks=MAX_BLOCKS, max_vertices=max_vertices)
    g.import_blocks(*to_dev(coords, tsdf, weight))
    g.extract(scope_all=True)
    g.gc()
    return sv, coords, tsdf, weight, g, g.status(check=False)


def test_crowded_segment_fills_first_and_a_fitted_pool_meshes():
    # every vertex in segment 0: its live count is the whole mesh's
    _, _, _, _, g, st = run(1 << 16)
    assert st["error"] == 0
    assert st["vertex_segments"] == NSEG and st["segment_capacity"] == (1 << 16) // NSEG
    live = st["vertex_slots"] - st["free_vertex_slots"]
    assert st["max_segment_live"] == live > 1000
    print(f"[pool] {live} vertices, all in one segment", flush=True)
    # a pool four times the mesh: segment 0 holds it exactly
    sv, coords, tsdf, weight, g, st = run(NSEG * live)
    assert st["error"] == 0 and st["max_segment_live"] == live
    o = oracle.OracleVolume(sv.voxel_m)
    o.import_blocks(coords, tsdf, weight)
    o.extract(scope_all=True)
    o.gc()
    compare_all(g, o)
    # one slot less per segment: the pool holds 4x the mesh minus 4, but
    # segment 0 cannot, and the documented error is raised
    _, _, _, _, g, st = run(NSEG * (live - 1))
    assert st["error"] == -4 and st["max_segment_live"] <= live - 1
