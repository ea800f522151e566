"""Batched forward + backward over independent volumes (one slot each) vs the
same steps volume by volume, vs the oracle, under HIP graph replay and under
every workgroup mapping.

Bar: the batch is an exact re-arrangement of the per-volume work, so the
vertex set (positions) and the TSDF gradient must agree bit for bit with
the plain per-volume path; against the oracle, each slot's vertex set and
counts are exact and its edge parameters t within 1e-5 voxel, and the
FP32 TSDF gradient is within 1e-4 relative (floor 1e-4 of the largest
magnitude) of the oracle's FP64 one."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from paper_1803_03949_amd import Volume, VmError
from paper_1803_03949_amd.binding import VM_BATCH_BACKWARD, VM_BATCH_FORWARD
from paper_1803_03949_amd.batch import (BatchMesher, PlainMesher, canonical_vertices,
                                        sphere_loss_grad)
from tests.gpu_compare import batch_vertices, compare_slot_vertices

pytestmark = pytest.mark.gpu

S = 0.008


def workload(n=6, lo=8, hi=400, seed=7):
    vols = scenes.batch_volumes(seed=seed, n=n, voxel_m=S, lo=lo, hi=hi)
    coords, ds, ws = [], [], []
    for v in vols:
        c, d, w = v.blocks()
        coords.append(c)
        ds.append(d)
        ws.append(w)
    tsdf = torch.from_numpy(np.concatenate(ds).reshape(-1, 512)).cuda()
    weight = torch.from_numpy(np.concatenate(ws).reshape(-1, 512)).cuda()
    centers = torch.tensor(np.stack([v.meta["center"] for v in vols]), dtype=torch.float32).cuda()
    radii = torch.tensor([v.meta["target_radius"] for v in vols], dtype=torch.float32).cuda()
    return vols, coords, tsdf, weight, centers, radii


def plain_for(coords, tsdf, weight, centers, radii):
    grads = [sphere_loss_grad(centers[i:i + 1], radii[i:i + 1]) for i in range(len(coords))]
    return PlainMesher(S, coords, tsdf, weight, grads)


def per_slot_vertices(m: BatchMesher):
    rows = canonical_vertices(m.pos, m.slot)
    return [rows[rows[:, 0] == k][:, 1:] for k in range(m.n_vol)]


def test_batch_matches_per_volume_path_bit_for_bit():
    vols, coords, tsdf, weight, centers, radii = workload()
    print(f"[batch] sizes {[len(c) for c in coords]}", flush=True)
    b = BatchMesher(S, coords, tsdf, weight, sphere_loss_grad(centers, radii))
    b.run()
    p = plain_for(coords, tsdf, weight, centers, radii)
    p.run()
    torch.cuda.synchronize()
    assert b.vol.status()["error"] == 0
    assert torch.equal(b.grad, p.grad())
    got = per_slot_vertices(b)
    for k, it in enumerate(p.items):
        want = canonical_vertices(it["pos"], it["slot"])[:, 1:]
        assert got[k].shape == want.shape and np.array_equal(got[k], want), k
    assert float(b.grad.abs().max()) > 0


def test_batch_gradient_matches_oracle():
    vols, coords, tsdf, weight, centers, radii = workload(n=3, lo=20, hi=150, seed=8)
    b = BatchMesher(S, coords, tsdf, weight, sphere_loss_grad(centers, radii))
    b.run()
    torch.cuda.synchronize()
    g = b.grad.cpu().numpy()
    bv = batch_vertices(b.vol)
    off = 0
    for k, v in enumerate(vols):
        c, d, w = v.blocks()
        o = oracle.OracleVolume(S)
        o.import_blocks(c, d, w)
        o.extract(scope_all=True)
        # the vertex set, counts and edge parameters t of the slot
        compare_slot_vertices(bv, k, o)
        pos = o.positions64()
        ctr, r = v.meta["center"], v.meta["target_radius"]
        dist = np.linalg.norm(pos - ctr, axis=1)
        dLdv = (2 * (dist - r) / dist)[:, None] * (pos - ctr)
        ref = o.grad_tsdf64(dLdv)
        oc = o.blocks()["coords"]
        idx = {tuple(x): i for i, x in enumerate(oc.tolist())}
        sel = np.array([idx[tuple(x)] for x in c.tolist()])
        want = ref[sel]
        got = g[off:off + len(c)]
        floor = 1e-4 * np.abs(want).max()
        assert np.all(np.abs(got - want) <= 1e-4 * np.abs(want) + floor), k
        off += len(c)


def test_graph_replays_match_eager():
    vols, coords, tsdf, weight, centers, radii = workload(n=5, seed=9)
    b = BatchMesher(S, coords, tsdf, weight, sphere_loss_grad(centers, radii))
    b.run()
    torch.cuda.synchronize()
    eager = b.grad.clone()
    eager_v = canonical_vertices(b.pos, b.slot)
    b.capture()
    p = plain_for(coords, tsdf, weight, centers, radii)
    for rep in range(3):
        b.grad.fill_(float("nan"))
        b.replay()
        torch.cuda.synchronize()
        assert torch.equal(b.grad, eager), rep
        assert np.array_equal(canonical_vertices(b.pos, b.slot), eager_v), rep
        p.run()  # unrelated eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("w", [2, 4, 8])
@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_every_mapping_gives_identical_bits(w, order):
    vols, coords, tsdf, weight, centers, radii = workload(n=4, seed=10)
    b = BatchMesher(S, coords, tsdf, weight, sphere_loss_grad(centers, radii))
    b.run()
    torch.cuda.synchronize()
    ref, ref_v = b.grad.clone(), canonical_vertices(b.pos, b.slot)
    for groups, bg in [(1, 1), (4, 2), (16, 8)]:
        b.set_launch(wave_group_size=w, wave_groups_per_cu=groups, block_groups_per_cu=bg,
                     item_groups_per_cu=groups, block_order=order)
        b.run()
        torch.cuda.synchronize()
        assert torch.equal(b.grad, ref), (groups, bg)
        assert np.array_equal(canonical_vertices(b.pos, b.slot), ref_v), (groups, bg)


def test_positions_are_the_downloaded_vertices():
    sv = scenes.sphere_volume(seed=1)
    c, d, w = sv.blocks()
    v = Volume(S, hash_log2=12, max_blocks=1024, max_vertices=1 << 16)
    v.import_blocks(*(torch.from_numpy(x).cuda() for x in (c, d.reshape(-1, 512), w.reshape(-1, 512))))
    v.extract(scope_all=True)
    pos, slot = v.positions()
    verts, _, _ = v.download(with_keys=False)
    live = canonical_vertices(pos, slot)
    assert np.all(live[:, 0] == 0)
    dv = verts.cpu().numpy().astype(np.float64)
    assert np.array_equal(live[:, 1:], dv[np.lexsort(dv.T[::-1])])


def test_batch_range_errors():
    b = Volume(S, hash_log2=12, max_blocks=64, max_vertices=1 << 12,
               batch_volumes=2)
    z = torch.zeros((1, 512), dtype=torch.float32, device="cuda")
    for slot, x in [(2, 0), (-1, 0), (0, 63), (0, -1)]:
        b.reset()
        b.import_batch(torch.tensor([slot], dtype=torch.int32, device="cuda"),
                       torch.tensor([[x, 0, 0]], dtype=torch.int32, device="cuda"), z, z)
        with pytest.raises(VmError, match="VM_ERR_RANGE"):
            b.status()
    # a batch takes no plain import and no depth frame
    b.reset()
    with pytest.raises(VmError, match="VM_ERR_ARG"):
        b.import_blocks(torch.zeros((1, 3), dtype=torch.int32, device="cuda"), z, z)


def test_extract_batch_entry_replays_its_graphs():
    """vm_extract_batch through the C ABI on a stream of the mesher's own, so
    that the library captures its forward and backward graphs on the first
    step and replays them after: every step gives the per-volume path's
    gradient bit for bit and the oracle's vertices, with other work between
    steps, and status and download read the replayed mesh."""
    vols, coords, tsdf, weight, centers, radii = workload(n=5, seed=12)
    print(f"[batch-entry] sizes {[len(c) for c in coords]}", flush=True)
    b = BatchMesher(S, coords, tsdf, weight, sphere_loss_grad(centers, radii))
    p = plain_for(coords, tsdf, weight, centers, radii)
    p.run()
    torch.cuda.synchronize()
    want = p.grad().clone()
    for rep in range(3):
        b.grad.fill_(float("nan"))
        b.step()
        torch.cuda.synchronize()
        assert torch.equal(b.grad, want), rep
        p.run()
        torch.cuda.synchronize()
    st = b.vol.status()
    assert st["error"] == 0 and st["blocks"] == b.n_blocks and st["dirty_blocks"] == b.n_blocks
    bv = batch_vertices(b.vol)
    for k, v in enumerate(vols):
        c, d, w = v.blocks()
        o = oracle.OracleVolume(S)
        o.import_blocks(c, d, w)
        o.extract(scope_all=True)
        compare_slot_vertices(bv, k, o)
    verts, tris, _ = b.vol.download()
    assert len(verts) == int((b.slot >= 0).sum()) and len(tris) == st["triangles"]


def test_extract_batch_rejects_bad_phases():
    """One phase per call: both bits, none or another value are refused
    before anything is enqueued."""
    vols, coords, tsdf, weight, centers, radii = workload(n=2, seed=13)
    b = BatchMesher(S, coords, tsdf, weight, sphere_loss_grad(centers, radii))
    for phase in (0, VM_BATCH_FORWARD | VM_BATCH_BACKWARD, 4):
        with pytest.raises(VmError, match="VM_ERR_ARG"):
            b.vol.extract_batch(b.io, phase, b.stream)
    b.step()
    torch.cuda.synchronize()
    assert b.vol.status()["error"] == 0
