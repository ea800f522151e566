"""Pins of the oracle's block collection (Eq. 1) and fusion (Eq. 2).

Closed forms: a fronto-parallel wall at constant depth seen from the
identity pose.  The collected blocks are then a full box whose z extent is
the depth band [D - mu, D + mu] and whose x/y extent is the view frustum at
the far end of the band; one frame into an empty volume stores the truncated
projective distance min((D - z)/s, mu) with weight 1; a second frame gives
the running average.
"""
import math

import numpy as np

import oracle
import scenes

S = 0.02          # voxel size (m)
MU = 4.0          # truncation (voxels)
D1, D2 = 1.013, 1.029


def wall_volume(*depths):
    vol = oracle.OracleVolume(S, MU)
    for D in depths:
        vol.integrate(scenes.plane_depth(D), scenes.K, np.eye(4, dtype=np.float32))
    return vol


def test_collected_blocks_form_the_frustum_box():
    vol = wall_volume(D1)
    got = vol.block_set("frame")
    B = 8 * S
    mu = MU * S
    zlo, zhi = math.floor((D1 - mu) / B), math.floor((D1 + mu) / B)
    fx, fy, cx, cy = scenes.K
    xlo = math.floor((0 - cx) / fx * (D1 + mu) / B)
    xhi = math.floor((scenes.WIDTH - 1 - cx) / fx * (D1 + mu) / B)
    ylo = math.floor((0 - cy) / fy * (D1 + mu) / B)
    yhi = math.floor((scenes.HEIGHT - 1 - cy) / fy * (D1 + mu) / B)
    want = {(x, y, z) for x in range(xlo, xhi + 1) for y in range(ylo, yhi + 1)
            for z in range(zlo, zhi + 1)}
    assert {tuple(b) for b in got.tolist()} == want
    assert vol.blocks()["coords"].shape[0] == len(want)


def expected_wall(vol, D):
    """FP64 closed form per voxel of every block: (in view, sdf)."""
    b = vol.blocks()
    c = b["coords"]
    l = np.arange(512)
    g = np.stack([8 * c[:, None, 0] + (l & 7), 8 * c[:, None, 1] + ((l >> 3) & 7),
                  8 * c[:, None, 2] + (l >> 6)], axis=-1).astype(np.float64) * S
    fx, fy, cx, cy = scenes.K
    z = g[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * g[..., 0] / z + cx
        v = fy * g[..., 1] / z + cy
    inside = (z > 0) & (u > -0.49) & (u < scenes.WIDTH - 0.51) & (v > -0.49) & (v < scenes.HEIGHT - 0.51)
    border = (z > 0) & ~inside & (u > -0.51) & (u < scenes.WIDTH - 0.49) & (v > -0.51) & (v < scenes.HEIGHT - 0.49)
    sdf = (D - z) / S
    return b, inside, border, sdf


def test_single_frame_stores_truncated_distance():
    vol = wall_volume(D1)
    b, inside, border, sdf = expected_wall(vol, D1)
    d, w = b["d"].astype(np.float64), b["w"]
    clear = inside & (np.abs(sdf + MU) > 1e-3)
    upd = clear & (sdf >= -MU)
    assert upd.sum() > 10000
    assert (w[upd] == 1).all()
    assert (w[clear & ~upd] == 0).all()
    assert (w[~inside & ~border] == 0).all()
    assert np.abs(d[upd] - np.minimum(sdf[upd], MU)).max() < 2e-5
    assert (d[w == 0] == 0).all()


def test_two_frames_running_average():
    vol = wall_volume(D1, D2)
    b, inside, border, _ = expected_wall(vol, D1)
    c = b["coords"]
    l = np.arange(512)
    z = (8 * c[:, None, 2] + (l >> 6)).astype(np.float64) * S
    sdf1, sdf2 = (D1 - z) / S, (D2 - z) / S
    both = inside & (sdf1 >= -MU + 1e-3) & (sdf2 >= -MU + 1e-3)
    assert both.sum() > 10000
    assert (b["w"][both] == 2).all()
    want = (np.minimum(sdf1, MU) + np.minimum(sdf2, MU)) / 2
    assert np.abs(b["d"][both] - want[both]).max() < 4e-5
    # the same frame twice leaves the distance unchanged, weight 2
    vol2 = wall_volume(D1, D1)
    b2 = vol2.blocks()
    b1 = wall_volume(D1).blocks()
    m = b1["w"] > 0
    assert (b2["d"][m] == b1["d"][m]).all() and (b2["w"][m] == 2).all()


def test_invalid_and_out_of_range_depth_is_ignored():
    depth = scenes.plane_depth(D1)
    depth[:, :320] = 0.0          # invalid
    depth[:240, 320:] = np.nan    # not finite
    vol = oracle.OracleVolume(S, MU)
    n = vol.integrate(depth, scenes.K, np.eye(4, dtype=np.float32), 0.4, 3.0)
    assert n > 0
    b = vol.blocks()
    # nothing left of the image centre column was collected
    fx, fy, cx, cy = scenes.K
    assert (b["coords"][:, 0] >= math.floor((320 - 1 - cx) / fx * (D1 + MU * S) / (8 * S))).all()
    # a depth range that excludes the wall collects nothing
    vol2 = oracle.OracleVolume(S, MU)
    assert vol2.integrate(scenes.plane_depth(D1), scenes.K, np.eye(4, dtype=np.float32), 1.5, 3.0) == 0


def test_pose_translation_shifts_the_collected_blocks():
    T = np.eye(4, dtype=np.float32)
    T[:3, 3] = [8 * S * 3, -8 * S * 2, 8 * S * 5]  # whole blocks
    a = {tuple(x) for x in wall_volume(D1).block_set("frame").tolist()}
    vol = oracle.OracleVolume(S, MU)
    vol.integrate(scenes.plane_depth(D1), scenes.K, T)
    b = {tuple(x) for x in vol.block_set("frame").tolist()}
    assert b == {(x + 3, y - 2, z + 5) for x, y, z in a}


def test_restricted_collection_matches_full_run_on_the_kept_blocks():
    """Collection and fusion of a block depend only on the depth frame and
    the block itself, so restricting collection to a sample of blocks gives
    those blocks bit for bit the TSDF and weights of the full run (and the
    absent ones stay absent)."""
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.008)
    frames = [seq.frame(k) for k in (0, 1)]
    full = oracle.OracleVolume(0.008)
    for k, f in enumerate(frames):
        full.integrate(f, scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
    fb = full.blocks()
    rng = np.random.default_rng(0)
    keep = fb["coords"][rng.choice(len(fb["coords"]), 24, replace=False)]
    have = {tuple(c) for c in fb["coords"].tolist()}
    absent = []
    for c in fb["coords"][rng.permutation(len(fb["coords"]))].tolist():
        for off in ((-2, 0, 0), (0, -2, 0), (0, 0, 2), (3, 3, 3)):
            n = (c[0] + off[0], c[1] + off[1], c[2] + off[2])
            if n not in have and len(absent) < 8:
                absent.append(n)
    sample = np.concatenate([keep, np.array(absent, np.int32)])
    part = oracle.OracleVolume(0.008)
    part.restrict(sample)
    for k, f in enumerate(frames):
        part.integrate(f, scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
    pb = part.blocks()
    assert {tuple(c) for c in pb["coords"].tolist()} == {tuple(c) for c in keep.tolist()}
    row = {tuple(c): i for i, c in enumerate(fb["coords"].tolist())}
    for i, c in enumerate(pb["coords"].tolist()):
        j = row[tuple(c)]
        assert np.array_equal(pb["d"][i].view(np.uint32), fb["d"][j].view(np.uint32))
        assert np.array_equal(pb["w"][i], fb["w"][j])
