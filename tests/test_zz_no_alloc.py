"""vm_create_volume_noalloc (workspace in the library's static per-device
array) against vm_create_volume (workspace in a caller buffer): the same
calls give the same blocks, cube types, vertices and triangles, on two
volumes in a row in the static workspace, the second one smaller and
meeting the first one's leftover contents."""
import numpy as np
import pytest

import scenes
from paper_1803_03949_amd import Volume, binding
from tests import meshutil
from tests.gpu_compare import gpu_blocks_sorted, gpu_live_vertices, gpu_triangle_keys, to_dev

pytestmark = pytest.mark.gpu


def run(vol, sv):
    coords, d, w = sv.blocks()
    vol.import_blocks(*to_dev(coords, d, w))
    vol.extract(scope_all=True)
    vol.refine()
    vol.gc()
    assert vol.status()["error"] == 0
    blocks = gpu_blocks_sorted(vol)
    keys, t, ref = gpu_live_vertices(vol)
    tri_keys, _, _ = gpu_triangle_keys(vol)
    return blocks, (keys, t, ref), meshutil.canonical_triangles(tri_keys)


def same(a, b):
    ba, va, ta = a
    bb, vb, tb = b
    assert (ba["coords"] == bb["coords"]).all()
    for k in ("d", "w", "prev", "cur"):
        assert np.array_equal(ba[k], bb[k]), k
    for x, y in zip(va, vb):
        assert x.shape == y.shape and np.array_equal(x, y)
    assert ta.shape == tb.shape and (ta == tb).all()
    return len(va[0]), len(ta)


@pytest.mark.parametrize("dims,cap", [((4, 4, 4), 512), ((2, 3, 2), 64)])
def test_noalloc_matches_caller_workspace(dims, cap):
    print(f"[noalloc] dims {dims} max_blocks {cap}", flush=True)
    sv = scenes.sphere_volume(seed=7, dims_blocks=dims, voxel_m=0.01,
                              radius=0.3 * 0.08 * min(dims), center=0.04 * np.asarray(dims),
                              jitter=0.004)
    kw = dict(hash_log2=12, max_blocks=cap, max_vertices=1 << 16)
    want = run(Volume(sv.voxel_m, **kw), sv)
    vol = Volume(sv.voxel_m, noalloc=True, **kw)
    assert vol.nbytes <= binding.NOALLOC_MAX_BYTES
    try:
        # the device's one static workspace is taken
        with pytest.raises(binding.VmError) as e:
            Volume(sv.voxel_m, noalloc=True, **kw)
        assert e.value.code == -1
        got = run(vol, sv)
        # and again on the same volume after a reset
        vol.reset()
        again = run(vol, sv)
    finally:
        vol.close()
    nv, nt = same(got, want)
    same(again, want)
    assert nv > 0 and nt > 0
