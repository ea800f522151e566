"""Full-size parity: the workloads at the sizes and launch configuration the
benchmark times.  The 8 mm sequence is replayed by the whole oracle and the
final states are compared in full; the 4 mm sequence with refinement (as a
pass after each extraction, and inside it) is checked on 50 sampled
neighbourhoods the oracle computes alone, plus properties that hold at any
size.

Sampling: collection and fusion of a block depend only on the depth frames
and on the block itself, and the mesh inside a block (cube types and their
history, the vertices the block owns with their counts, the triangles of its
cubes) depends only on the blocks of its 3x3x3 neighbourhood.  So the
oracle, restricted to the neighbourhoods of a few sampled blocks, replays
the whole sequence cheaply and gives exact expected values for the sampled
blocks; every expected value comes from the oracle run on the same inputs.

Bar: bit-exact block membership, cube types, vertex sets, reference counts
and triangle connectivity; TSDF, weights and t within 1e-5 voxel."""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import scenes
from paper_1803_03949_amd import Volume, key_to_edge
from tests.gpu_compare import compare_all, to_dev
from tests.sampling import check_invariants, check_samples, neighbourhood, sample_blocks, state

pytestmark = pytest.mark.gpu


def gpu_state(g):
    b = g.export_blocks()
    blocks = {k: (b[k].cpu().numpy() if k != "coords" else b[k]) for k in b}
    v = g.export_vertices()
    ref = v["ref"].cpu().numpy()
    live = ref > 0
    _, tris, keys = g.download()
    return state(blocks, key_to_edge(v["keys"].cpu().numpy()[live]),
                 v["t"].cpu().numpy()[live], ref[live],
                 key_to_edge(keys.cpu().numpy())[tris.cpu().numpy()])


def render(seq, n):
    with ProcessPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(seq.frame, range(n)))


def test_room_sequence_8mm_full_size():
    """100 frames, 640x480, 8 mm, 2^20 hash slots, integrate+extract+gc per
    frame, the benchmark's volume and launch configuration, against the
    unrestricted oracle replaying the whole sequence: every block, cube
    type, vertex and triangle of the final state."""
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.008)
    frames = render(seq, 100)
    print("[full] room 8 mm: GPU", flush=True)
    g = Volume(0.008, hash_log2=20, max_blocks=1 << 17, max_vertices=1 << 23)
    depth = to_dev(np.stack(frames))[0]
    for k in range(100):
        g.integrate(depth[k], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        g.extract()
        g.gc()
    assert g.status()["error"] == 0
    check_invariants(gpu_state(g))
    print("[full] room 8 mm: oracle, whole sequence", flush=True)
    o = oracle.OracleVolume(0.008, threads=min(16, os.cpu_count() or 1), keep_fusion=False)
    for k in range(100):
        o.integrate(frames[k], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        o.extract()
        o.gc()
        if (k + 1) % 20 == 0:
            print(f"[full] room 8 mm: oracle frame {k + 1}", flush=True)
    info = compare_all(g, o)
    print(f"[full] room 8 mm: {info}", flush=True)
    assert info["nv"] > 10 ** 6


_FRAMES_4MM = {}


@pytest.mark.parametrize("mode", ["pass", "inside"])
def test_room_sequence_4mm_refine_full_size(mode):
    """500 frames, 4 mm, holes, refinement at every extraction (a refinement
    pass after it, or inside it: VM_EXTRACT_REFINE), 2^22 hash slots, the
    benchmark's volume configuration."""
    seq = scenes.room_sequence(seed=3, n_frames=500, voxel_m=0.004, holes=True)
    if "frames" not in _FRAMES_4MM:
        _FRAMES_4MM["frames"] = render(seq, 500)
    frames = _FRAMES_4MM["frames"]
    inside = mode == "inside"
    print(f"[full] room 4 mm + refine ({mode}): GPU", flush=True)
    g = Volume(0.004, hash_log2=22, max_blocks=1 << 19, max_vertices=1 << 24)
    depth = to_dev(np.stack(frames))[0]
    for k in range(500):
        g.integrate(depth[k], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        g.extract(refine=inside)
        if not inside:
            g.refine()
        g.gc()
    state = gpu_state(g)
    check_invariants(state)
    assert g.totals()["refined_cubes"] > 0
    samples = sample_blocks(state[1], np.random.default_rng(22), 40, 10)
    print(f"[full] room 4 mm ({mode}): oracle on {len(samples)} sampled neighbourhoods", flush=True)
    o = oracle.OracleVolume(0.004, threads=min(16, os.cpu_count() or 1), keep_fusion=False)
    o.restrict(neighbourhood(samples.tolist()))
    for k in range(500):
        o.integrate(frames[k], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        o.extract(refine=inside)
        if not inside:
            o.refine()
        o.gc()
    check_samples(state, o, samples)
