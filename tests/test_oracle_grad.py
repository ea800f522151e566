"""Pins of the oracle's FP64 backward pass against FP64 central finite
differences, with the mesh connectivity held fixed.

Vertex positions depend on the fused TSDF through the edge interpolation
(Sec. V-C) and the fused TSDF depends on the depth frame through the running
average of Eq. (2); the loss is the squared distance of every vertex to a
slightly larger target sphere."""
import numpy as np
import pytest

import oracle
import scenes

S = 0.01


def sphere_setup(with_frame):
    sv = scenes.sphere_volume(seed=11, dims_blocks=(2, 2, 2), voxel_m=S, radius=0.05,
                              center=np.full(3, 0.08), jitter=0.005)
    vol = oracle.OracleVolume(S, 4.0)
    coords, d = scenes.dense_to_blocks(sv.tsdf)
    vol.import_blocks(coords, d, np.ones_like(d))
    depth = pose = None
    if with_frame:
        c = sv.meta["center"]
        pose = scenes.look_at(c + np.array([0.02, -0.30, 0.12]), c).astype(np.float32)
        sc = scenes.Scene([(c + np.array([0.0, 0.0, 0.002]), 0.0505)], [], None)
        depth = sc.render(pose.astype(np.float64), scenes.pixel_rays(), None, 0.1, 5.0)
        vol.integrate(depth, scenes.K, pose, 0.1, 5.0)
    vol.extract(scope_all=True)
    return vol, sv, depth


def loss_and_grad(pos, c, rt):
    r = np.linalg.norm(pos - c, axis=1)
    e = r - rt
    return float((e * e).sum()), (2 * e / r)[:, None] * (pos - c)


def test_tsdf_gradient_matches_finite_differences():
    vol, sv, _ = sphere_setup(False)
    c, rt = sv.meta["center"], sv.meta["radius"] + 0.003
    pos = vol.positions64()
    _, dL_dv = loss_and_grad(pos, c, rt)
    g = vol.grad_tsdf64(dL_dv)
    coords = vol.blocks()["coords"]
    nz = np.argwhere(g != 0)
    assert len(nz) > 100
    rng = np.random.default_rng(0)
    h = 1e-6
    scale = np.abs(g).max()
    for bi, l in nz[rng.choice(len(nz), 40, replace=False)]:
        gx = 8 * coords[bi, 0] + (l & 7)
        gy = 8 * coords[bi, 1] + ((l >> 3) & 7)
        gz = 8 * coords[bi, 2] + (l >> 6)
        lp, _ = loss_and_grad(vol.positions64((gx, gy, gz), h), c, rt)
        lm, _ = loss_and_grad(vol.positions64((gx, gy, gz), -h), c, rt)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[bi, l]) <= 1e-6 * scale + 1e-6 * abs(fd), (gx, gy, gz, fd, g[bi, l])
    # a voxel no vertex depends on has zero gradient, and FD agrees
    zero = np.argwhere(g == 0)[0]
    bi, l = zero
    v = (8 * coords[bi, 0] + (l & 7), 8 * coords[bi, 1] + ((l >> 3) & 7), 8 * coords[bi, 2] + (l >> 6))
    lp, _ = loss_and_grad(vol.positions64(v, h), c, rt)
    lm, _ = loss_and_grad(vol.positions64(v, -h), c, rt)
    assert lp == lm


def test_depth_gradient_matches_finite_differences():
    vol, sv, depth = sphere_setup(True)
    c, rt = sv.meta["center"], sv.meta["radius"] + 0.003
    pos = vol.positions64()
    _, dL_dv = loss_and_grad(pos, c, rt)
    g1 = vol.grad_tsdf64(dL_dv)
    H, W = depth.shape
    g0, gD = vol.grad_fusion64(g1, H, W)
    fu = vol.fused()
    assert len(fu["pixel"]) > 300
    # closed form of the weight factor: imported voxels had weight 1 and pass
    # half their gradient to the old TSDF; voxels of blocks the frame newly
    # allocated had weight 0 and pass none
    coords = vol.blocks()["coords"]
    idx = {tuple(b): i for i, b in enumerate(coords.tolist())}
    seen = set()
    for (x, y, z), w0 in zip(fu["voxel"].tolist(), fu["w0"]):
        bi = idx[(x // 8, y // 8, z // 8)]
        l = (x % 8) + 8 * (y % 8) + 64 * (z % 8)
        inside = all(0 <= q < 16 for q in (x, y, z))
        assert w0 == (1.0 if inside else 0.0)
        assert g0[bi, l] == (g1[bi, l] * 0.5 if inside else 0.0)
        seen.add(inside)
    assert seen == {True, False}
    nzp = np.flatnonzero(gD)
    assert len(nzp) > 50
    rng = np.random.default_rng(1)
    h = 1e-7
    scale = np.abs(gD).max()
    for p in rng.choice(nzp, 30, replace=False):
        lp, _ = loss_and_grad(vol.positions64_depth(p, h), c, rt)
        lm, _ = loss_and_grad(vol.positions64_depth(p, -h), c, rt)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gD.flat[p]) <= 1e-6 * scale + 1e-5 * abs(fd), (p, fd, gD.flat[p])
