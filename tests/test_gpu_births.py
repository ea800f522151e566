"""Vertex birth frames (vm_download_births) vs the oracle, exactly.

Frames count integrations and imports from 1; a vertex's birth frame is the
frame of the pass at whose end its count last became positive.  The GPU
frees a vertex when its count drops to zero and creates a new one when the
edge is needed again, the oracle keeps it until its GC and revives it: both
give the stamp of the pass in which the count became positive again, which
the sequences below (extract + gc, and extract + refine + gc) exercise."""
import numpy as np
import pytest

import oracle
import scenes
from paper_1803_03949_amd import Volume, key_to_edge
from tests.gpu_compare import to_dev

pytestmark = pytest.mark.gpu


def gpu_births_in_key_order(g):
    _, _, keys = g.download()
    b = g.download_births().cpu().numpy()
    k = key_to_edge(keys.cpu().numpy())
    order = np.lexsort(k.T[::-1])
    return k[order], b[order]


def run(seq, frames, refine):
    g = Volume(seq.voxel_m, hash_log2=16, max_blocks=1 << 14, max_vertices=1 << 20)
    o = oracle.OracleVolume(seq.voxel_m, 4.0, 0.5)
    for k in frames:
        depth = seq.frame(k)
        g.integrate(to_dev(depth)[0], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        o.integrate(depth, scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        g.extract(refine=refine == "fused")
        o.extract(refine=refine == "fused")
        if refine is True:
            g.refine()
            o.refine()
        g.gc()
        o.gc()
    gk, gb = gpu_births_in_key_order(g)
    ok = o.vertices()["keys"]
    assert gk.shape == ok.shape and (gk == ok).all()
    ob = o.births()
    assert (gb == ob).all(), np.flatnonzero(gb != ob)[:10]
    return gb


def test_room_sequence_births():
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.03)
    b = run(seq, range(8), refine=False)
    assert b.min() == 1 and len(np.unique(b)) > 3


def test_refinement_sequence_births():
    seq = scenes.room_sequence(seed=3, n_frames=500, voxel_m=0.03, holes=True)
    b = run(seq, range(0, 12, 2), refine=True)
    assert len(np.unique(b)) > 3


def test_refining_extraction_births():
    seq = scenes.room_sequence(seed=3, n_frames=500, voxel_m=0.03, holes=True)
    b = run(seq, range(0, 12, 2), refine="fused")
    assert len(np.unique(b)) > 3


def test_batched_import_births():
    sv = scenes.sphere_volume(seed=1)
    c, d, w = sv.blocks()
    g = Volume(0.008, hash_log2=12, max_blocks=1024, max_vertices=1 << 16)
    g.import_blocks(*to_dev(c, d, w))
    g.extract(scope_all=True)
    g.download()
    assert (g.download_births().cpu().numpy() == 1).all()
