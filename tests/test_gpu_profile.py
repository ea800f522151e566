"""Kernel timing (vm_profile, vm_profile_mask, vm_profile_read): each
profiled launch is counted once with its own start-to-end time, a mask
limits the records to its kernels, and profiling leaves results unchanged."""
import time

import numpy as np
import pytest
import torch

import scenes
from paper_1803_03949_amd import Volume
from tests.gpu_compare import to_dev

pytestmark = pytest.mark.gpu

FRAMES = (0, 2, 4, 6)


def run(profile, kernels=None):
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.03)
    g = Volume(seq.voxel_m, hash_log2=16, max_blocks=1 << 14, max_vertices=1 << 20)
    depth = [to_dev(seq.frame(k))[0] for k in FRAMES]
    if profile:
        g.profile(True, kernels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d, k in zip(depth, FRAMES):
        g.integrate(d, scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        g.extract()
        g.gc()
    torch.cuda.synchronize()
    wall_ms = 1e3 * (time.perf_counter() - t0)
    prof = g.profile_read() if profile else {}
    g.profile(False)
    return g, prof, wall_ms


def test_every_kernel_counted_once_per_launch_with_its_own_time():
    print("[profile] all kernels", flush=True)
    g, prof, wall_ms = run(True)
    n = len(FRAMES)
    for k in ("collect", "fuse", "dirty", "classify", "vertices"):
        launches, ms = prof[k]
        assert launches == n, (k, launches)
        assert 0.0 < ms < wall_ms, (k, ms, wall_ms)
    assert sum(ms for _, ms in prof.values()) < wall_ms


def test_mask_records_only_its_kernels_and_results_are_unchanged():
    print("[profile] vertices only", flush=True)
    g, prof, _ = run(True, ["vertices"])
    assert set(prof) == {"vertices"} and prof["vertices"][0] == len(FRAMES)
    ref, _, _ = run(False)
    assert g.status()["triangles"] == ref.status()["triangles"]
    assert g.totals() == ref.totals()
