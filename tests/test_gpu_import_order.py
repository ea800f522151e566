"""Imports number new blocks in input order: into an empty volume input row
i becomes pool row i, and a later import appends its new blocks after the
existing ones, again in input order, while blocks already present keep
their rows.  The frame list follows the input order too.  The mesh of the
imported volume still matches the oracle's."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from paper_1803_03949_amd import Volume
from tests.gpu_compare import compare_all, to_dev

pytestmark = pytest.mark.gpu

S = 0.008


def sphere_blocks():
    v = scenes.sphere_volume(seed=1, dims_blocks=(6, 5, 4), voxel_m=S, radius=0.12)
    return v.blocks()


def test_import_rows_become_pool_rows():
    c, d, w = sphere_blocks()
    perm = np.random.default_rng(3).permutation(len(c))
    c, d, w = c[perm], d[perm], w[perm]
    g = Volume(S, hash_log2=12, max_blocks=1 << 10, max_vertices=1 << 16)
    g.import_blocks(*to_dev(c, d, w))
    assert np.array_equal(g.export_blocks()["coords"], c)
    assert np.array_equal(g.block_list("frame"), c)
    assert np.array_equal(g.lookup(to_dev(c)[0]).cpu().numpy(), np.arange(len(c)))
    o = oracle.OracleVolume(S)
    o.import_blocks(c, d, w)
    g.extract()
    o.extract()
    compare_all(g, o)


def test_second_import_appends_new_blocks_in_order():
    c, d, w = sphere_blocks()
    n = len(c)
    first = np.arange(0, n, 2)
    rng = np.random.default_rng(4)
    # the second import mixes blocks already present (new data) and new ones
    second = rng.permutation(np.concatenate([np.arange(1, n, 2), first[::3]]))
    g = Volume(S, hash_log2=12, max_blocks=1 << 10, max_vertices=1 << 16)
    o = oracle.OracleVolume(S)
    g.import_blocks(*to_dev(c[first], d[first], w[first]))
    o.import_blocks(c[first], d[first], w[first])
    d2 = d[second] * np.float32(0.5)
    g.import_blocks(*to_dev(c[second], d2, w[second]))
    o.import_blocks(c[second], d2, w[second])
    rows = g.lookup(to_dev(c)[0]).cpu().numpy()
    assert np.array_equal(rows[first], np.arange(len(first)))
    fresh = [k for k in second if k % 2 == 1]
    assert np.array_equal(rows[fresh], len(first) + np.arange(len(fresh)))
    assert np.array_equal(g.block_list("frame"), c[second])
    # pending: the first import's blocks, then the second's new ones
    assert np.array_equal(g.block_list("pending"), np.concatenate([c[first], c[fresh]]))
    g.extract()
    o.extract()
    compare_all(g, o)


def test_batch_import_rows_are_consecutive():
    vols = scenes.batch_volumes(seed=7, n=3, voxel_m=S, lo=8, hi=60)
    coords, ds, ws, slots = [], [], [], []
    for k, v in enumerate(vols):
        c, d, w = v.blocks()
        coords.append(c)
        ds.append(d)
        ws.append(w)
        slots.append(np.full(len(c), k, np.int32))
    c = np.concatenate(coords)
    g = Volume(S, hash_log2=12, max_blocks=len(c), max_vertices=1 << 16, batch_volumes=3)
    rows = torch.empty(len(c), dtype=torch.int32, device="cuda")
    g.import_batch(to_dev(np.concatenate(slots))[0], to_dev(c)[0],
                   *to_dev(np.concatenate(ds), np.concatenate(ws)), rows)
    torch.cuda.synchronize()
    assert np.array_equal(rows.cpu().numpy(), np.arange(len(c)))
    assert g.status()["error"] == 0
