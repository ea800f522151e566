"""The sampling argument behind the full-size GPU parity tests, checked on
the oracle alone: a run restricted to the neighbourhoods of sampled blocks
reproduces a full run's state on those blocks exactly (membership, TSDF,
weights, cube types and history, owned vertices with t and counts, the
triangles of their cubes), with and without refinement."""
import numpy as np
import pytest

import oracle
import scenes
from tests.sampling import (check_invariants, check_samples, neighbourhood, oracle_state,
                            sample_blocks)


@pytest.mark.parametrize("refine", [False, True])
def test_restricted_run_reproduces_sampled_blocks(refine):
    seq = scenes.room_sequence(seed=3 if refine else 2, n_frames=100, voxel_m=0.008,
                               holes=refine)
    ks = (0, 1, 2)
    frames = [seq.frame(k) for k in ks]

    def run(o):
        for k, f in zip(ks, frames):
            o.integrate(f, scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
            o.extract()
            if refine:
                o.refine()
            o.gc()

    full = oracle.OracleVolume(0.008)
    run(full)
    fs = oracle_state(full)
    check_invariants(fs)
    samples = sample_blocks(fs[1], np.random.default_rng(5), 12, 4)
    part = oracle.OracleVolume(0.008)
    part.restrict(neighbourhood(samples.tolist()))
    run(part)
    check_samples(fs, part, samples)
    if refine:
        assert full.blocks()["cur"].size and len(fs[2]) > 0
    # planted mistakes in the full state are caught
    b, rows, verts, tris = fs
    present = [tuple(s) for s in samples.tolist() if tuple(s) in rows]
    owned = [k for k in verts if (k[0] // 8, k[1] // 8, k[2] // 8) in present]
    assert owned
    bad = dict(verts)
    bad[owned[0]] = (bad[owned[0]][0] + 1e-3, bad[owned[0]][1])
    with pytest.raises(AssertionError):
        check_samples((b, rows, bad, tris), part, samples)
    bad = dict(verts)
    del bad[owned[-1]]
    with pytest.raises(AssertionError):
        check_samples((b, rows, bad, tris), part, samples)
    lo = np.floor_divide(tris[:, :, :3].min(axis=1), 8)
    hit = np.nonzero((lo == np.array(present[0])).all(axis=1))[0]
    if len(hit):
        with pytest.raises(AssertionError):
            check_samples((b, rows, verts, np.delete(tris, hit[0], axis=0)), part, samples)
