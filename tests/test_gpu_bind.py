"""Caller-owned TSDF storage (vm_bind_tsdf): imports then copy nothing.
The batched step with bound tensors gives the same bits as with copies;
a bound plain volume meshes as the oracle does; imports must pass the bound
tensors, and a row that would not land on its own pool row is refused;
fusion writes the bound tensors; unbinding restores copying imports."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from paper_1803_03949_amd import Volume, VmError
from paper_1803_03949_amd.batch import BatchMesher, PlainMesher, canonical_vertices, sphere_loss_grad
from tests.gpu_compare import compare_all, to_dev

pytestmark = pytest.mark.gpu

S = 0.008


def batch_inputs(seed=11, n=5):
    vols = scenes.batch_volumes(seed=seed, n=n, voxel_m=S, lo=8, hi=300)
    coords, ds, ws = [], [], []
    for v in vols:
        c, d, w = v.blocks()
        coords.append(c)
        ds.append(d)
        ws.append(w)
    tsdf = torch.from_numpy(np.concatenate(ds)).cuda()
    weight = torch.from_numpy(np.concatenate(ws)).cuda()
    centers = torch.tensor(np.stack([v.meta["center"] for v in vols]), dtype=torch.float32).cuda()
    radii = torch.tensor([v.meta["target_radius"] for v in vols], dtype=torch.float32).cuda()
    return coords, tsdf, weight, centers, radii


def test_bound_batch_gives_the_bits_of_copying_imports():
    coords, tsdf, weight, centers, radii = batch_inputs()
    print(f"[bind] sizes {[len(c) for c in coords]}", flush=True)
    ref = BatchMesher(S, coords, tsdf, weight, sphere_loss_grad(centers, radii), zero_copy=False)
    ref.run()
    b = BatchMesher(S, coords, tsdf, weight, sphere_loss_grad(centers, radii))
    b.capture()
    for rep in range(2):
        b.grad.fill_(float("nan"))
        b.replay()
        torch.cuda.synchronize()
        assert b.vol.status()["error"] == 0
        assert torch.equal(b.grad, ref.grad), rep
        assert np.array_equal(canonical_vertices(b.pos, b.slot),
                              canonical_vertices(ref.pos, ref.slot)), rep
    p = PlainMesher(S, coords, tsdf, weight,
                    [sphere_loss_grad(centers[i:i + 1], radii[i:i + 1]) for i in range(len(coords))])
    p.run()
    torch.cuda.synchronize()
    assert torch.equal(p.grad(), ref.grad)


def test_bound_plain_volume_matches_oracle_and_checks_rows():
    v = scenes.sphere_volume(seed=1, dims_blocks=(5, 4, 4), voxel_m=S, radius=0.1)
    c, d, w = v.blocks()
    n = len(c)
    g = Volume(S, hash_log2=12, max_blocks=n, max_vertices=1 << 16)
    td, tw = to_dev(d, w)
    g.bind_tsdf(td, tw)
    g.import_blocks(to_dev(c)[0], td, tw)
    o = oracle.OracleVolume(S)
    o.import_blocks(c, d, w)
    g.extract()
    o.extract()
    compare_all(g, o)
    # other tensors than the bound ones are refused
    with pytest.raises(VmError):
        g.import_blocks(to_dev(c)[0], td.clone(), tw)
    # the same rows again land on their own pool rows: accepted
    g.import_blocks(to_dev(c)[0], td, tw)
    assert g.status()["error"] == 0
    # new blocks of a second import would land after the first import's
    # rows, not on their own: refused
    g.reset()
    g.import_blocks(to_dev(c[: n // 2])[0], td, tw)
    assert g.status()["error"] == 0
    g.import_blocks(to_dev(c[n // 2:])[0], td, tw)
    st = g.status(check=False)
    assert st["error"] == -8  # VM_ERR_RANGE
    perm = np.roll(np.arange(n), 1)
    # unbound again: a copying import of the permuted rows works
    g.bind_tsdf(None, None)
    g.reset()
    g.import_blocks(*to_dev(c[perm], d[perm], w[perm]))
    g.extract()
    o2 = oracle.OracleVolume(S)
    o2.import_blocks(c[perm], d[perm], w[perm])
    o2.extract()
    compare_all(g, o2)


def test_fusion_writes_the_bound_tensors():
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.03)
    B = 1 << 12
    g = Volume(0.03, hash_log2=14, max_blocks=B, max_vertices=1 << 18)
    td = torch.zeros((B, 512), dtype=torch.float32, device="cuda")
    tw = torch.zeros_like(td)
    g.bind_tsdf(td, tw)
    o = oracle.OracleVolume(0.03)
    for k in range(2):
        depth = seq.frame(k)
        g.integrate(to_dev(depth)[0], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        o.integrate(depth, scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        g.extract()
        o.extract()
    compare_all(g, o)
    b = g.export_blocks()
    m = len(b["coords"])
    assert torch.equal(b["d"], td[:m]) and torch.equal(b["w"], tw[:m])
    assert float(tw[:m].max()) > 0
