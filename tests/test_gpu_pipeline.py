"""Frames pipelined as the benchmark runs them: each frame's triangle pass on
a side stream (vm_extract_mesh_split) while the next frame is collected and
fused, the next extraction waiting for it.  The mesh after every joined
frame equals the oracle's, frame after frame, on the room sequence with
holes (many blocks created while triangles are being written)."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from paper_1803_03949_amd import Volume
from tests.gpu_compare import compare_all, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("voxel", [0.03, 0.008])
def test_pipelined_frames_match_oracle(voxel):
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=voxel, holes=True)
    print(f"[pipeline] voxel {voxel}", flush=True)
    g = Volume(voxel, hash_log2=18, max_blocks=1 << 15, max_vertices=1 << 21)
    o = oracle.OracleVolume(voxel)
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    frames = list(range(0, 40, 4)) if voxel > 0.01 else list(range(0, 12, 4))
    for n, k in enumerate(frames):
        depth = seq.frame(k)
        g.integrate(to_dev(depth)[0], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        if n:
            main.wait_stream(side)
        g.extract(tri_stream=side)
        g.gc()
        o.integrate(depth, scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        o.extract()
        if n % 3 == 2:
            # the next frame is collected and fused while this one's
            # triangles are written; then the mesh is joined and compared
            main.wait_stream(side)
            compare_all(g, o)
    main.wait_stream(side)
    compare_all(g, o)
