"""The oracle's vertex normals, pinned to closed forms (CPU only).

Reading (the paper keeps a normal per vertex, Sec. IV, without saying how
it is formed): the TSDF gradient by central differences over observed
voxels (one-sided where a neighbour is unobserved or unallocated),
interpolated along the vertex's edge at t and normalised; it points to
increasing TSDF.  Pins: a linear field has an exact gradient under both
difference formulas, so every normal is the field's direction, also next to
unobserved voxels holding garbage; on a sampled sphere the normals follow
the radial direction far more closely than the owner voxel's gradient alone
would; normals agree in sign with the oracle's outward triangle
orientation."""
import numpy as np
import pytest

import oracle
import scenes
from scenes import dense_to_blocks


def linear_volume(a, b, n=16, unobserved_from_x=None):
    # dense arrays are indexed (z, y, x)
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d = (a[0] * xx + a[1] * yy + a[2] * zz + b).astype(np.float32)
    w = np.ones_like(d)
    if unobserved_from_x is not None:
        d[:, :, unobserved_from_x:] = 100.0  # garbage that must never be read
        w[:, :, unobserved_from_x:] = 0.0
    c, db = dense_to_blocks(d)
    _, wb = dense_to_blocks(w)
    o = oracle.OracleVolume(0.01)
    o.import_blocks(c, db, wb)
    o.extract(scope_all=True)
    return o


@pytest.mark.parametrize("a", [(0.3, -0.5, 0.8), (1.0, 0.0, 0.0), (-0.2, 0.7, 0.1)])
def test_linear_field_normals_are_its_direction(a):
    o = linear_volume(a, -(np.dot(a, (7.3, 8.1, 6.6))))
    n, ln = o.normals64()
    assert len(n) > 50
    want = np.asarray(a) / np.linalg.norm(a)
    assert np.abs(n - want).max() < 1e-6
    assert np.allclose(ln, np.linalg.norm(a), rtol=1e-6)


def test_one_sided_differences_next_to_unobserved_voxels():
    a = (0.9, 0.3, -0.4)
    o = linear_volume(a, -(np.dot(a, (5.5, 8.2, 7.7))), unobserved_from_x=9)
    keys = o.vertices()["keys"]
    n, _ = o.normals64()
    # vertices whose gradient stencil touches x = 9 exist and are exact too
    assert (keys[:, 0] + (keys[:, 3] == 0) == 8).any()
    want = np.asarray(a) / np.linalg.norm(a)
    assert np.abs(n - want).max() < 1e-6


def test_sphere_normals_follow_the_radius():
    sv = scenes.sphere_volume(seed=3, dims_blocks=(8, 8, 8), voxel_m=0.008, radius=0.20)
    c, d, w = sv.blocks()
    o = oracle.OracleVolume(0.008)
    o.import_blocks(c, d, w)
    o.extract(scope_all=True)
    n, ln = o.normals64()
    pos = o.positions64()
    radial = pos - sv.meta["center"]
    radial /= np.linalg.norm(radial, axis=1, keepdims=True)
    ang = np.arccos(np.clip((n * radial).sum(1), -1, 1))
    # the owner voxel's gradient alone would be off by up to about one voxel
    # of arc, 0.008/0.2 = 0.04 rad; the interpolated one is far closer
    assert ang.max() < 4e-3, ang.max()
    assert np.all(ln > 0.9)


def test_normals_agree_with_outward_triangles():
    sv = scenes.sphere_volume(seed=4, dims_blocks=(8, 8, 8), voxel_m=0.008, radius=0.20)
    c, d, w = sv.blocks()
    o = oracle.OracleVolume(0.008)
    o.import_blocks(c, d, w)
    o.extract(scope_all=True)
    n, _ = o.normals64()
    verts, tris = o.download()
    v = verts.astype(np.float64)
    face = np.cross(v[tris[:, 1]] - v[tris[:, 0]], v[tris[:, 2]] - v[tris[:, 0]])
    face /= np.linalg.norm(face, axis=1, keepdims=True)
    # vertex order of the download is the key order of normals64
    for j in range(3):
        assert ((n[tris[:, j]] * face).sum(1) > 0.5).all()
