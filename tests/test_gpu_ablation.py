"""The paper's two vertex-sharing schemes (Sec. V-C), run as an ablation
beside edge ownership: both must initialise exactly one vertex per edge the
dirty cubes' types use, with the same edge parameter t, as the oracle's
vertex set and t on a from-scratch extraction; and they must agree with each
other over an incremental sequence.  Integer state exact, t bit-exact (the
same FP32 formula)."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from paper_1803_03949_amd import Volume
from tests.gpu_compare import to_dev

pytestmark = pytest.mark.gpu


def fresh_state(g):
    n = g.cfg.max_blocks * 3 * 512
    slot = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    t = torch.zeros(n, dtype=torch.float32, device="cuda")
    counter = torch.zeros(1, dtype=torch.int32, device="cuda")
    return slot, t, counter


def edge_keys(g, slot):
    coords = g.export_blocks()["coords"]
    e = np.flatnonzero(slot.cpu().numpy() >= 0)
    blk, axis, l = e // 1536, (e // 512) % 3, e % 512
    c = coords[blk]
    return np.stack([8 * c[:, 0] + (l & 7), 8 * c[:, 1] + ((l >> 3) & 7), 8 * c[:, 2] + (l >> 6),
                     axis], axis=1), e


@pytest.mark.parametrize("scheme", [0, 1])
def test_schemes_match_the_oracle_vertex_set(scheme):
    sv = scenes.sphere_volume(seed=1)
    c, d, w = sv.blocks()
    g = Volume(0.008, hash_log2=12, max_blocks=1024, max_vertices=1 << 16)
    g.import_blocks(*to_dev(c, d, w))
    g.extract(scope_all=True)
    slot, t, counter = fresh_state(g)
    g.sharing_ablation(scheme, slot, t, counter)
    torch.cuda.synchronize()
    keys, e = edge_keys(g, slot)
    order = np.lexsort(keys.T[::-1])
    o = oracle.OracleVolume(0.008)
    o.import_blocks(c, d, w)
    o.extract(scope_all=True)
    ov = o.vertices()
    assert keys.shape == ov["keys"].shape and (keys[order] == ov["keys"]).all()
    assert (t.cpu().numpy()[e][order] == ov["t"]).all()
    n = int(counter.item())
    assert n == len(e) and np.array_equal(np.sort(slot.cpu().numpy()[e]), np.arange(n))


def test_schemes_agree_over_a_sequence():
    seq = scenes.room_sequence(seed=2, n_frames=100, voxel_m=0.03)
    g = Volume(seq.voxel_m, hash_log2=16, max_blocks=1 << 13, max_vertices=1 << 20)
    states = [fresh_state(g), fresh_state(g)]
    for k in range(0, 18, 3):
        g.integrate(to_dev(seq.frame(k))[0], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        g.extract()
        g.gc()
        for scheme, st in enumerate(states):
            g.sharing_ablation(scheme, *st)
    torch.cuda.synchronize()
    (s0, t0, c0), (s1, t1, c1) = states
    m0, m1 = s0 >= 0, s1 >= 0
    assert torch.equal(m0, m1) and int(m0.sum()) > 1000
    assert torch.equal(t0[m0], t1[m1])
    assert int(c0.item()) == int(c1.item()) == int(m0.sum())
