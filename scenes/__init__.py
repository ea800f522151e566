"""Seeded synthetic inputs for the volumetric meshing path.

The paper evaluates on recorded RGB-D sequences (ICL-NUIM, TUM RGB-D and the
Zhou-Koltun scenes) that are not available here.  These generators stand in
for them with the same sensor model (640x480 depth, Kinect-like intrinsics
fx = fy = 525, cx = 319.5, cy = 239.5 and a depth-dependent noise) at the
paper's fine resolutions (8 mm, 4 mm).  No item of those datasets is
reproduced.

This module produces inputs only: analytic signed distances sampled on a
lattice, depth maps ray-cast from analytic scenes, camera poses.  It holds
none of the meshing method's arithmetic and is shared by the GPU tests and
the CPU oracle alike.  Everything is computed in FP64 with
``numpy.random.default_rng(seed)`` and cast to FP32 at the end.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FX = FY = 525.0
CX, CY = 319.5, 239.5
WIDTH, HEIGHT = 640, 480
K = (FX, FY, CX, CY)


# ----------------------------------------------------------------------------
# dense lattices and their block decomposition
# ----------------------------------------------------------------------------

def dense_to_blocks(dense: np.ndarray, origin_block=(0, 0, 0)):
    """Split a dense (Z, Y, X) voxel array (each extent a multiple of 8) into
    8^3 blocks.  Returns (coords (n,3) int32, values (n,512)) with block
    coordinates in x, y, z order and each block's voxels in x-fastest order."""
    Z, Y, X = dense.shape
    assert X % 8 == 0 and Y % 8 == 0 and Z % 8 == 0
    bz, by, bx = Z // 8, Y // 8, X // 8
    v = dense.reshape(bz, 8, by, 8, bx, 8).transpose(0, 2, 4, 1, 3, 5).reshape(bz * by * bx, 512)
    zz, yy, xx = np.meshgrid(np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    coords = np.stack([xx.ravel() + origin_block[0], yy.ravel() + origin_block[1],
                       zz.ravel() + origin_block[2]], axis=1).astype(np.int32)
    return coords, np.ascontiguousarray(v)


def lattice_points(dims_vox, voxel_m, origin_vox=(0, 0, 0)):
    """World coordinates (FP64) of lattice corners g*s, arrays shaped (Z, Y, X)."""
    X, Y, Z = dims_vox
    gx = (np.arange(X) + origin_vox[0]) * voxel_m
    gy = (np.arange(Y) + origin_vox[1]) * voxel_m
    gz = (np.arange(Z) + origin_vox[2]) * voxel_m
    return np.meshgrid(gz, gy, gx, indexing="ij")[::-1]  # x, y, z each (Z, Y, X)


# ----------------------------------------------------------------------------
# analytic signed distances
# ----------------------------------------------------------------------------

def sdf_sphere(x, y, z, center, r):
    return np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2) - r


def sdf_box(x, y, z, center, half, yaw):
    """Box with half extents `half`, rotated by `yaw` about +z."""
    c, s = math.cos(yaw), math.sin(yaw)
    px, py, pz = x - center[0], y - center[1], z - center[2]
    lx = c * px + s * py
    ly = -s * px + c * py
    qx, qy, qz = np.abs(lx) - half[0], np.abs(ly) - half[1], np.abs(pz) - half[2]
    outside = np.sqrt(np.maximum(qx, 0) ** 2 + np.maximum(qy, 0) ** 2 + np.maximum(qz, 0) ** 2)
    inside = np.minimum(np.maximum(qx, np.maximum(qy, qz)), 0.0)
    return outside + inside


def truncate(sdf_m, voxel_m, trunc_vox=4.0):
    """Sampled TSDF in voxel units: clip(sdf/s, -trunc, trunc), as FP32."""
    return np.clip(sdf_m / voxel_m, -trunc_vox, trunc_vox).astype(np.float32)


# ----------------------------------------------------------------------------
# sphere volumes (single and batched)
# ----------------------------------------------------------------------------

@dataclass
class DenseVolume:
    voxel_m: float
    dims_blocks: tuple        # (bx, by, bz)
    tsdf: np.ndarray          # (Z, Y, X) float32, voxel units
    weight: np.ndarray        # (Z, Y, X) float32
    meta: dict = field(default_factory=dict)

    def blocks(self):
        c, d = dense_to_blocks(self.tsdf)
        _, w = dense_to_blocks(self.weight)
        return c, d, w


def sphere_volume(seed=1, dims_blocks=(8, 8, 8), voxel_m=0.008, radius=0.30,
                  center=None, jitter=0.02, trunc_vox=4.0) -> DenseVolume:
    """Sphere sampled directly as a TSDF with unit weight on a block lattice
    starting at the origin.  Default: 8x8x8 blocks at 8 mm, r = 0.30 m, centre
    0.256 m per axis plus a seeded offset in +-2 cm."""
    rng = np.random.default_rng(seed)
    bx, by, bz = dims_blocks
    dims_vox = (8 * bx, 8 * by, 8 * bz)
    if center is None:
        center = np.full(3, 0.256)
    center = np.asarray(center, np.float64) + rng.uniform(-jitter, jitter, 3)
    x, y, z = lattice_points(dims_vox, voxel_m)
    tsdf = truncate(sdf_sphere(x, y, z, center, radius), voxel_m, trunc_vox)
    return DenseVolume(voxel_m, (bx, by, bz), tsdf, np.ones_like(tsdf),
                       dict(center=center, radius=radius))


def batch_volumes(seed=5, n=64, voxel_m=0.008, lo=50, hi=20000, trunc_vox=4.0,
                  max_blocks=None):
    """Independent sphere volumes with log-uniform block counts in [lo, hi].
    Each is a bx*by*bz block box with bx = by = round(N^(1/3)) and
    bz = round(N/(bx*by)); the sphere radius is 0.586 of the smallest extent
    (the single-sphere case's 0.30/0.512) and its centre sits mid-box plus a
    seeded offset in +-2 cm."""
    rng = np.random.default_rng(seed)
    vols = []
    for _ in range(n):
        N = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        if max_blocks is not None:
            N = min(N, max_blocks)
        b = max(1, int(round(N ** (1.0 / 3.0))))
        bzz = max(1, int(round(N / (b * b))))
        extent = np.array([8 * b, 8 * b, 8 * bzz], np.float64) * voxel_m
        r = 0.586 * float(extent.min())
        center = extent / 2 + rng.uniform(-0.02, 0.02, 3)
        x, y, z = lattice_points((8 * b, 8 * b, 8 * bzz), voxel_m)
        tsdf = truncate(sdf_sphere(x, y, z, center, r), voxel_m, trunc_vox)
        vols.append(DenseVolume(voxel_m, (b, b, bzz), tsdf, np.ones_like(tsdf),
                                dict(center=center, radius=r, target_radius=r + voxel_m)))
    return vols


# ----------------------------------------------------------------------------
# cameras and ray casting
# ----------------------------------------------------------------------------

def look_at(position, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """4x4 camera-to-world pose; camera x right, y down, z forward."""
    p = np.asarray(position, np.float64)
    f = np.asarray(target, np.float64) - p
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    T = np.eye(4)
    T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = r, d, f, p
    return T


def pixel_rays(W=WIDTH, H=HEIGHT, K=K):
    fx, fy, cx, cy = K
    u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    return np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], axis=-1)  # (H, W, 3)


def _ray_sphere(o, d, a, c, r):
    """Nearest positive hit of rays o + lam*d (d given as 3 component arrays,
    a = |d|^2) with a sphere; inf where missed."""
    ocx, ocy, ocz = o[0] - c[0], o[1] - c[1], o[2] - c[2]
    b = d[0] * ocx + d[1] * ocy + d[2] * ocz
    cc = ocx * ocx + ocy * ocy + ocz * ocz - r * r
    disc = b * b - a * cc
    ok = disc >= 0
    sq = np.sqrt(np.where(ok, disc, 0.0))
    l0 = (-b - sq) / a
    l1 = (-b + sq) / a
    near = np.where(l0 > 1e-9, l0, np.where(l1 > 1e-9, l1, np.inf))
    return np.where(ok, near, np.inf)


def _ray_box(o, d, center, half, yaw, interior=False):
    """Slab test against a box rotated by yaw about +z; inf where missed.
    interior=True returns the exit distance of rays starting inside."""
    c, s = math.cos(yaw), math.sin(yaw)
    px, py, pz = o[0] - center[0], o[1] - center[1], o[2] - center[2]
    lo = (c * px + s * py, -s * px + c * py, pz)
    ld = (c * d[0] + s * d[1], -s * d[0] + c * d[1], d[2])
    tmin = tmax = None
    with np.errstate(divide="ignore", invalid="ignore"):
        for i in range(3):
            t1 = (-half[i] - lo[i]) / ld[i]
            t2 = (half[i] - lo[i]) / ld[i]
            lo_t, hi_t = np.fmin(t1, t2), np.fmax(t1, t2)
            tmin = lo_t if tmin is None else np.fmax(tmin, lo_t)
            tmax = hi_t if tmax is None else np.fmin(tmax, hi_t)
    if interior:
        return np.where(tmax > 1e-9, tmax, np.inf)
    hit = (tmax >= tmin) & (tmax > 1e-9)
    near = np.where(tmin > 1e-9, tmin, tmax)
    return np.where(hit, near, np.inf)


def kinect_noise(z, rng):
    sigma = 0.0012 + 0.0019 * (z - 0.4) ** 2
    return z + rng.normal(0.0, 1.0, z.shape) * sigma


@dataclass
class Scene:
    spheres: list   # (center(3), r)
    boxes: list     # (center(3), half(3), yaw)
    room: tuple | None  # (lo(3), hi(3)) interior, or None

    def render(self, T_cw, rays, rng=None, min_depth=0.4, max_depth=3.0):
        """z-depth (FP32, metres; 0 = invalid) seen from camera pose T_cw."""
        R, o = T_cw[:3, :3], T_cw[:3, 3]
        shape = rays.shape[:-1]
        rx, ry, rz = (rays[..., i].ravel() for i in range(3))
        d = tuple(R[i, 0] * rx + R[i, 1] * ry + R[i, 2] * rz for i in range(3))
        a = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
        lam = np.full(rx.shape, np.inf)
        for c, r in self.spheres:
            lam = np.minimum(lam, _ray_sphere(o, d, a, np.asarray(c), r))
        for c, h, yaw in self.boxes:
            # only rays through the box's bounding sphere can hit it
            near = np.isfinite(_ray_sphere(o, d, a, np.asarray(c), float(np.linalg.norm(h)) * 1.001))
            if near.any():
                sub = tuple(x[near] for x in d)
                lam[near] = np.minimum(lam[near], _ray_box(o, sub, np.asarray(c), np.asarray(h), yaw))
        if self.room is not None:
            lo, hi = (np.asarray(v, np.float64) for v in self.room)
            lam = np.minimum(lam, _ray_box(o, d, (lo + hi) / 2, (hi - lo) / 2, 0.0, interior=True))
        lam = lam.reshape(shape)
        z = lam  # rays have unit camera-z, so the ray parameter is the z-depth
        if rng is not None:
            z = np.where(np.isfinite(z), kinect_noise(np.where(np.isfinite(z), z, 0.0), rng), z)
        z = np.where(np.isfinite(z) & (z >= min_depth) & (z <= max_depth), z, 0.0)
        return z.astype(np.float32)

    def sdf(self, x, y, z):
        parts = [sdf_sphere(x, y, z, c, r) for c, r in self.spheres]
        parts += [sdf_box(x, y, z, c, h, yaw) for c, h, yaw in self.boxes]
        out = parts[0]
        for p in parts[1:]:
            out = np.minimum(out, p)
        return out


# ----------------------------------------------------------------------------
# the analytic room sequence
# ----------------------------------------------------------------------------

@dataclass
class RoomSequence:
    voxel_m: float
    scene: Scene
    poses: list            # 4x4 FP32 camera-to-world
    seed: int
    holes: bool
    min_depth: float = 0.4
    max_depth: float = 3.0

    def __len__(self):
        return len(self.poses)

    def frame(self, k: int) -> np.ndarray:
        """Depth frame k (FP32 H x W); deterministic per (seed, k)."""
        rng = np.random.default_rng([self.seed, 1000 + k])
        rays = pixel_rays()
        depth = self.scene.render(self.poses[k].astype(np.float64), rays, rng,
                                  self.min_depth, self.max_depth)
        if self.holes:
            depth = drop_discs(depth, rng, 0.10)
        return depth


def drop_discs(depth, rng, fraction, rmin=4, rmax=32):
    H, W = depth.shape
    mask = np.zeros((H, W), bool)
    vv, uu = np.mgrid[0:H, 0:W]
    while mask.mean() < fraction:
        cu, cv = rng.uniform(0, W), rng.uniform(0, H)
        r = rng.uniform(rmin, rmax)
        mask |= (uu - cu) ** 2 + (vv - cv) ** 2 <= r * r
    out = depth.copy()
    out[mask] = 0.0
    return out


def room_sequence(seed=2, n_frames=100, voxel_m=0.008, holes=False) -> RoomSequence:
    """A 4 x 4 x 3 m room with 10 spheres (r in [0.1, 0.5] m) and 10 yawed
    boxes (sides in [0.1, 0.8] m) seen along one smooth closed camera loop."""
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(0.8, 1.2, 2)
    phi0 = rng.uniform(0, 2 * math.pi)
    centre = np.array([2.0, 2.0, 1.5])
    poses, path = [], []
    for k in range(n_frames):
        th = phi0 + 2 * math.pi * k / n_frames
        p = centre + np.array([a * math.cos(th), b * math.sin(th), 0.2 * math.sin(2 * th)])
        tgt = np.array([2.0, 2.0, 1.0]) + 0.8 * np.array([math.cos(th + math.pi / 3),
                                                           math.sin(th + math.pi / 3), 0.0])
        poses.append(look_at(p, tgt).astype(np.float32))
        path.append(p)
    dense_path = []
    for k in range(720):
        th = 2 * math.pi * k / 720
        dense_path.append(centre + np.array([a * math.cos(th), b * math.sin(th), 0.2 * math.sin(2 * th)]))
    dense_path = np.array(dense_path)
    px, py, pz = dense_path[:, 0], dense_path[:, 1], dense_path[:, 2]

    spheres, boxes = [], []
    while len(spheres) < 10:
        r = rng.uniform(0.1, 0.5)
        c = rng.uniform([r, r, r], [4 - r, 4 - r, 3 - r])
        if sdf_sphere(px, py, pz, c, r).min() >= 0.4:
            spheres.append((c, r))
    while len(boxes) < 10:
        half = rng.uniform(0.1, 0.8, 3) / 2
        yaw = rng.uniform(0, math.pi / 2)
        ext = np.linalg.norm(half[:2])
        c = rng.uniform([ext, ext, half[2]], [4 - ext, 4 - ext, 3 - half[2]])
        if sdf_box(px, py, pz, c, half, yaw).min() >= 0.4:
            boxes.append((c, half, yaw))
    scene = Scene(spheres, boxes, ((0.0, 0.0, 0.0), (4.0, 4.0, 3.0)))
    return RoomSequence(voxel_m, scene, poses, seed, holes)


# ----------------------------------------------------------------------------
# the differentiable-extraction scene: sphere plus five boxes, one frame
# ----------------------------------------------------------------------------

@dataclass
class GradScene:
    volume: DenseVolume
    depth: np.ndarray
    pose: np.ndarray
    scene: Scene
    target: Scene


def grad_scene(seed=4, dims_blocks=(16, 16, 16), voxel_m=0.008, trunc_vox=4.0,
               box_count=5) -> GradScene:
    rng = np.random.default_rng(seed)
    ext = np.array(dims_blocks, np.float64) * 8 * voxel_m
    mid = ext / 2
    sc = mid + rng.uniform(-0.02, 0.02, 3)
    r = 0.30 * float(ext.min()) / 1.024
    boxes = []
    for _ in range(box_count):
        c = rng.uniform(mid - 0.212 * ext.min() / 1.024, mid + 0.212 * ext.min() / 1.024)
        half = rng.uniform(0.08, 0.25, 3) / 2
        yaw = rng.uniform(0, math.pi / 2)
        boxes.append((c, half, yaw))
    scene = Scene([(sc, r)], boxes, None)
    shifts = rng.uniform(-0.005, 0.005, (box_count, 3))
    target = Scene([(sc, r + 0.01)],
                   [(c + sh, h * 1.02, yaw) for (c, h, yaw), sh in zip(boxes, shifts)], None)
    x, y, z = lattice_points(tuple(8 * b for b in dims_blocks), voxel_m)
    tsdf = truncate(scene.sdf(x, y, z), voxel_m, trunc_vox)
    vol = DenseVolume(voxel_m, tuple(dims_blocks), tsdf, np.ones_like(tsdf), dict(radius=r))
    cam = np.array([mid[0], -0.9 * ext[1] / 1.024, 0.9 * ext[2] / 1.024])
    pose = look_at(cam, np.array([mid[0], mid[1], 0.45 * ext[2] / 1.024])).astype(np.float32)
    depth = scene.render(pose.astype(np.float64), pixel_rays(), rng, 0.1, 10.0)
    return GradScene(vol, depth, pose, scene, target)


def plane_depth(depth_m: float, W=WIDTH, H=HEIGHT) -> np.ndarray:
    """A fronto-parallel wall at constant camera depth."""
    return np.full((H, W), depth_m, np.float32)
