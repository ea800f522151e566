"""Comparison of the GPU library's state with the oracle's, after canonical
sorting (hash insertion order and pool slots are not deterministic)."""
from __future__ import annotations

import numpy as np
import torch

from paper_1803_03949_amd import key_to_edge
from tests import meshutil

TOL = 1e-5  # voxel units, for TSDF, weights and edge parameters


def gpu_blocks_sorted(gvol):
    b = gvol.export_blocks()
    c = b["coords"]
    order = np.lexsort(c.T[::-1])
    out = {"coords": c[order]}
    for k in ("d", "w", "prev", "cur"):
        out[k] = b[k].cpu().numpy()[order]
    return out


def compare_blocks(gvol, ovol, types=True):
    g = gpu_blocks_sorted(gvol)
    o = ovol.blocks()
    assert g["coords"].shape == o["coords"].shape, (g["coords"].shape, o["coords"].shape)
    assert (g["coords"] == o["coords"]).all(), "hash membership differs"
    dd = np.abs(g["d"].astype(np.float64) - o["d"]).max(initial=0)
    dw = np.abs(g["w"].astype(np.float64) - o["w"]).max(initial=0)
    assert dd <= TOL and dw <= TOL, (dd, dw)
    if types:
        assert (g["cur"] == o["cur"]).all(), int((g["cur"] != o["cur"]).sum())
        assert (g["prev"] == o["prev"]).all(), int((g["prev"] != o["prev"]).sum())
    return dict(max_d=float(dd), max_w=float(dw), bitexact_d=bool(dd == 0))


def gpu_live_vertices(gvol):
    v = gvol.export_vertices()
    ref = v["ref"].cpu().numpy()
    live = ref > 0
    keys = key_to_edge(v["keys"].cpu().numpy()[live])
    t = v["t"].cpu().numpy()[live]
    ref = ref[live]
    order = np.lexsort(keys.T[::-1])
    return keys[order], t[order], ref[order]


def compare_vertices(gvol, ovol):
    gk, gt, gr = gpu_live_vertices(gvol)
    o = ovol.vertices(live_only=True)
    assert gk.shape == o["keys"].shape, (gk.shape, o["keys"].shape)
    assert (gk == o["keys"]).all(), "vertex set differs"
    assert (gr == o["ref"]).all(), "reference counts differ"
    dt = np.abs(gt.astype(np.float64) - o["t"]).max(initial=0)
    assert dt <= TOL, dt
    return dict(nv=len(gk), max_t=float(dt))


def gpu_triangle_keys(gvol):
    verts, tris, keys = gvol.download()
    k = key_to_edge(keys.cpu().numpy())
    t = tris.cpu().numpy()
    assert (t >= 0).all() and (t < len(k)).all()
    return k[t], verts.cpu().numpy(), t


def compare_triangles(gvol, ovol):
    gk, _, _ = gpu_triangle_keys(gvol)
    ok = ovol.triangles()
    assert gk.shape == ok.shape, (gk.shape, ok.shape)
    a = meshutil.canonical_triangles(gk)
    b = meshutil.canonical_triangles(ok)
    assert (a == b).all(), "triangle connectivity differs"
    return dict(nt=len(gk))


def compare_all(gvol, ovol):
    info = compare_blocks(gvol, ovol)
    info.update(compare_vertices(gvol, ovol))
    info.update(compare_triangles(gvol, ovol))
    return info


def to_dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def batch_vertices(gvol):
    """Live vertices of a batched volume from its vertex pool: slot, edge
    (gx, gy, gz, axis) in the slot's own frame, t and count."""
    from paper_1803_03949_amd.binding import SLOT_SPAN
    v = gvol.export_vertices()
    ref = v["ref"].cpu().numpy()
    live = ref > 0
    edges = key_to_edge(v["keys"].cpu().numpy()[live])
    slot = (edges[:, 0] // 8 + 8192) // SLOT_SPAN
    edges[:, 0] -= 8 * (SLOT_SPAN * slot - 8192)
    return slot, edges, v["t"].cpu().numpy()[live], ref[live]


def compare_slot_vertices(bv, k, ovol):
    """Slot k of batch_vertices(...) against an oracle volume holding that
    slot's blocks alone: vertex set and counts exact, t within TOL."""
    slot, edges, t, ref = bv
    mine = slot == k
    e, tk, rk = edges[mine], t[mine], ref[mine]
    order = np.lexsort(e.T[::-1])
    e, tk, rk = e[order], tk[order], rk[order]
    o = ovol.vertices(live_only=True)
    assert e.shape == o["keys"].shape, (k, e.shape, o["keys"].shape)
    assert (e == o["keys"]).all(), f"vertex set of slot {k} differs"
    assert (rk == o["ref"]).all(), f"reference counts of slot {k} differ"
    dt = np.abs(tk.astype(np.float64) - o["t"]).max(initial=0)
    assert dt <= TOL, (k, dt)
    return dict(nv=int(len(e)), max_t=float(dt))
