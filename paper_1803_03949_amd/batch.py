"""Batched forward + backward over many independent volumes.

All volumes live in one batched library volume (one slot each), so every
kernel of the sequence -- reset, import, classification, vertices,
positions, backward -- runs once over the blocks of all of them, on a grid
sized to the device rather than to one volume.  The forward and the
backward are the library's vm_extract_batch phases, each a HIP graph the
library captures once and replays; the whole step, the caller's loss
included, can also be captured into one torch graph (the library then
launches its kernels into that capture).

The loss is the caller's: a function from (positions, slot of each vertex
pool entry) to dL/dpositions made of elementwise torch operations, so that
it can sit inside the graph too.  `sphere_loss_grad` is the one used by the
benchmark: squared distance of every vertex to a per-volume target sphere.

`PlainMesher` runs the same steps volume by volume, each in a volume of its
own: the per-volume path the batch is measured against.
"""
from __future__ import annotations

import json
import math
import os
import time
import zlib

import numpy as np
import torch

from .binding import SLOT_SPAN, VM_BATCH_BACKWARD, VM_BATCH_FORWARD, Volume


def sphere_loss_grad(centers: torch.Tensor, radii: torch.Tensor):
    """dL/dp for L = sum over live vertices of (|p - c_k| - r_k)^2, with
    (c_k, r_k) the target sphere of the vertex's volume k.  Elementwise
    operations only (the distance as two hypot calls), so the function can
    be graph-captured and every entry goes through the same operations
    whatever the pool size.  Entries with
    slot -1 (no vertex, position 0) index an extra sphere of radius 0 at the
    origin, whose gradient at the origin is 0."""
    dev = centers.device
    zero = torch.zeros(1, dtype=torch.float32, device=dev)
    centers = torch.cat([centers.reshape(-1, 3).float(), zero.expand(1, 3)]).contiguous()
    radii = torch.cat([radii.reshape(-1).float(), zero]).contiguous()
    rows = centers.shape[0]

    def grad(pos: torch.Tensor, slot: torch.Tensor, out: torch.Tensor):
        k = slot.remainder(rows)  # -1 -> the extra sphere
        d = pos - centers.index_select(0, k)
        dist = torch.hypot(torch.hypot(d[:, 0], d[:, 1]), d[:, 2]).clamp_min_(1e-30)
        scale = (dist - radii.index_select(0, k)).div_(dist).mul_(2.0)
        return torch.mul(d, scale[:, None], out=out)

    return grad


def sphere_loss(pos: torch.Tensor, slot: torch.Tensor, centers, radii) -> float:
    """The loss value itself (FP64, outside any graph)."""
    live = slot >= 0
    p = pos[live].double()
    k = slot[live].long()
    d = torch.linalg.norm(p - centers.double()[k], dim=1) - radii.double()[k]
    return float((d * d).sum())


def vertex_capacity(n_blocks: int) -> int:
    """A generous vertex pool size for a volume of n_blocks blocks holding a
    sphere-like surface: 64 per block plus 8192 (the 64 workload volumes
    hold 15 vertices per block on average, at most 102 per block in volumes
    of a few blocks, which the constant covers)."""
    return 64 * n_blocks + 8192


def fitted_capacity(status: dict, margin: float = 1.25) -> int:
    """Vertex pool size from a volume's status after a forward: every
    segment gets `margin` times the fullest one's live vertices plus 64, so
    the positions export and the caller's loss walk about `margin` times
    the live vertices rather than the generous bound.  A later forward
    whose surface outgrows it raises VM_ERR_VERTEX_POOL_FULL (refit then)."""
    per = int(math.ceil(margin * status["max_segment_live"])) + 64
    return status["vertex_segments"] * per


class BatchMesher:
    """Forward (import, extract everything, positions) and backward (dL/dTSDF)
    of many volumes as one batch.

    coords: list of (n_i, 3) int32 block coordinates, 0 <= x <= 62;
    tsdf, weight: (sum n_i, 512) FP32 device tensors in the same order.
    With zero_copy (the default) the volume uses tsdf and weight as its own
    storage (`Volume.bind_tsdf`): every import numbers the blocks in input
    order into the emptied volume, so row i of the tensors is pool row i and
    nothing is copied; the tensors must stay alive and unchanged between
    runs, or change only through the caller's own updates between them.
    After `run()` (eager) or `replay()` (graph), `grad` holds dL/dTSDF in the
    input order, `pos`/`slot` the vertex positions per pool entry."""

    def __init__(self, voxel_m: float, coords: list, tsdf: torch.Tensor, weight: torch.Tensor,
                 loss_grad, trunc_vox: float = 4.0, zero_copy: bool = True,
                 max_vertices: int | None = None):
        """max_vertices: the vertex pool size; None fits it to the workload
        with one probing forward at the generous bound (`fitted_capacity`)."""
        self.n_vol = len(coords)
        sizes = [int(len(c)) for c in coords]
        self.sizes = sizes
        N = sum(sizes)
        self.n_blocks = N
        if max_vertices is None:
            probe = BatchMesher(voxel_m, coords, tsdf, weight, loss_grad, trunc_vox, zero_copy,
                                max_vertices=vertex_capacity(N))
            probe.forward()
            max_vertices = fitted_capacity(probe.vol.status())
            del probe
        V = max_vertices
        hash_log2 = max(12, int(math.ceil(math.log2(max(2 * N, 2)))))
        self.vol = Volume(voxel_m, trunc_vox=trunc_vox, hash_log2=hash_log2, max_blocks=N,
                          max_vertices=V, batch_volumes=self.n_vol)
        dev = self.vol.device
        c = np.concatenate([np.asarray(x, np.int32).reshape(-1, 3) for x in coords])
        assert c[:, 0].min() >= 0 and c[:, 0].max() <= SLOT_SPAN - 2
        self.coords = torch.from_numpy(c).to(dev)
        self.slots = torch.from_numpy(np.repeat(np.arange(self.n_vol, dtype=np.int32),
                                                sizes)).to(dev)
        self.tsdf = tsdf
        self.weight = weight
        if zero_copy:
            self.vol.bind_tsdf(tsdf, weight)
        self.rows = torch.empty(N, dtype=torch.int32, device=dev)
        self.pos = torch.empty((V, 3), dtype=torch.float32, device=dev)
        self.slot = torch.empty(V, dtype=torch.int32, device=dev)
        self.dpos = torch.zeros((V, 3), dtype=torch.float32, device=dev)
        self.grad = torch.empty((N, 512), dtype=torch.float32, device=dev)
        self.loss_grad = loss_grad
        self.graph = None
        self.io = self.vol.batch_io(self.slots, self.coords, tsdf, weight, self.rows, self.pos,
                                    self.slot, self.dpos, self.grad)
        # the library captures its graphs on a stream of its own caller's
        # (the legacy default stream cannot be captured); default priority
        self.stream = torch.cuda.Stream(device=dev)

    def run(self, stream=None):
        """The whole step on `stream` (default: the current one): the
        library's forward, the caller's loss gradient, the library's
        backward.  On the legacy default stream, or under a capture, the
        library's phases are plain launches; elsewhere they are its graphs."""
        v = self.vol
        cur = torch.cuda.current_stream(v.device) if stream is None else stream
        v.extract_batch(self.io, VM_BATCH_FORWARD, cur)
        with torch.cuda.stream(cur):
            self.loss_grad(self.pos, self.slot, self.dpos)
        v.extract_batch(self.io, VM_BATCH_BACKWARD, cur)

    def forward(self):
        """The library's forward alone, on the mesher's stream, joined."""
        cur = torch.cuda.current_stream(self.vol.device)
        self.stream.wait_stream(cur)
        self.vol.extract_batch(self.io, VM_BATCH_FORWARD, self.stream)
        cur.wait_stream(self.stream)

    def step(self):
        """`run` on the mesher's own stream, joined to the current stream on
        both sides: the library replays its own forward and backward graphs,
        the loss gradient runs between them."""
        cur = torch.cuda.current_stream(self.vol.device)
        self.stream.wait_stream(cur)
        self.run(self.stream)
        cur.wait_stream(self.stream)

    def capture(self):
        """Capture `run` in a HIP graph (after one eager warm-up run)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        torch.cuda.synchronize()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def set_launch(self, **kw):
        """Change the workgroup mapping (drops a captured graph)."""
        self.vol.set_launch(**kw)
        self.graph = None


class PlainMesher:
    """The same step volume by volume, each in its own plain volume."""

    def __init__(self, voxel_m: float, coords: list, tsdf: torch.Tensor, weight: torch.Tensor,
                 loss_grads: list, trunc_vox: float = 4.0, zero_copy: bool = True):
        """Each volume's vertex pool fitted as the batch's is (one probing
        forward per volume at the generous bound)."""
        self.vols, self.items = [], []
        off = 0
        for i, c in enumerate(coords):
            n = int(len(c))
            hash_log2 = max(12, int(math.ceil(math.log2(max(2 * n, 2)))))
            probe = Volume(voxel_m, trunc_vox=trunc_vox, hash_log2=hash_log2, max_blocks=n,
                           max_vertices=vertex_capacity(n))
            cdev = torch.from_numpy(np.asarray(c, np.int32).reshape(-1, 3)).to(probe.device)
            probe.import_blocks(cdev, tsdf[off:off + n].contiguous(),
                                weight[off:off + n].contiguous())
            probe.extract(scope_all=True)
            V = fitted_capacity(probe.status())
            del probe
            vol = Volume(voxel_m, trunc_vox=trunc_vox, hash_log2=hash_log2, max_blocks=n,
                         max_vertices=V)
            dev = vol.device
            self.items.append(dict(
                coords=torch.from_numpy(np.asarray(c, np.int32).reshape(-1, 3)).to(dev),
                tsdf=tsdf[off:off + n], weight=weight[off:off + n],
                rows=torch.empty(n, dtype=torch.int32, device=dev),
                pos=torch.empty((V, 3), dtype=torch.float32, device=dev),
                slot=torch.empty(V, dtype=torch.int32, device=dev),
                dpos=torch.zeros((V, 3), dtype=torch.float32, device=dev),
                grad=torch.empty((n, 512), dtype=torch.float32, device=dev),
                loss_grad=loss_grads[i]))
            if zero_copy:
                vol.bind_tsdf(self.items[-1]["tsdf"], self.items[-1]["weight"])
            self.vols.append(vol)
            off += n

    def run(self):
        """Volume after volume on the current stream."""
        for v, it in zip(self.vols, self.items):
            v.reset()
            v.import_batch(None, it["coords"], it["tsdf"], it["weight"], it["rows"])
            v.extract(scope_all=True)
            v.positions(it["pos"], it["slot"])
            it["loss_grad"](it["pos"], it["slot"], it["dpos"])
            v.extract_backward_slots(it["dpos"], it["rows"], it["grad"])

    def grad(self) -> torch.Tensor:
        return torch.cat([it["grad"] for it in self.items])


def canonical_vertices(pos: torch.Tensor, slot: torch.Tensor) -> np.ndarray:
    """Live vertices as (slot, x, y, z) rows sorted lexicographically: a
    pool-order-independent view of the forward result."""
    live = (slot >= 0).cpu().numpy()
    p = pos.cpu().numpy()[live]
    s = slot.cpu().numpy()[live].astype(np.float64)
    rows = np.concatenate([s[:, None], p.astype(np.float64)], axis=1)
    order = np.lexsort(rows.T[::-1])
    return rows[order]


# ----------------------------------------------------------------------------
# autotuner
# ----------------------------------------------------------------------------

def default_space():
    """Workgroup mappings tried by `autotune`."""
    out = []
    for w in (2, 4, 8):
        for groups in (8 // w * 4, 8 // w * 8):  # 16 or 32 waves per CU
            for bg in (2, 4, 8):
                for order in (0, 1, 2, 3):
                    out.append(dict(wave_group_size=w, wave_groups_per_cu=max(1, groups),
                                    block_groups_per_cu=bg, item_groups_per_cu=8,
                                    block_order=order))
    return out


def _time_replays(m: BatchMesher, reps: int) -> float:
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        start.record()
        m.replay()
        stop.record()
        stop.synchronize()
        times.append(start.elapsed_time(stop))
    return float(np.median(times))


def cache_path() -> str:
    return os.environ.get("VOXMESH_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "voxmesh", "tune.json"))


def workload_key(m: BatchMesher) -> str:
    name = torch.cuda.get_device_name(m.vol.device)
    crc = zlib.crc32(np.asarray(m.sizes, np.int64).tobytes())
    return f"{name}|vols={m.n_vol}|blocks={m.n_blocks}|sizes={crc:08x}"


def autotune(m: BatchMesher, space=None, reps: int = 10, use_cache: bool = True,
             log=None) -> dict:
    """Time every mapping of `space` on graph replays of `m`, check that each
    gives the same bits (gradient in input order, canonical vertex set) as
    the first, and leave `m` captured with the fastest.  The winner is cached
    in a JSON file keyed by device and workload."""
    key = workload_key(m)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        m.set_launch(**cache[key]["launch"])
        m.capture()
        return dict(cache[key], cached=True)
    space = space or default_space()
    ref_grad = ref_verts = None
    results = []
    for cfg in space:
        m.set_launch(**cfg)
        m.capture()
        m.replay()
        torch.cuda.synchronize()
        g = m.grad.clone()
        verts = canonical_vertices(m.pos, m.slot)
        if ref_grad is None:
            ref_grad, ref_verts = g, verts
        same = bool(torch.equal(g, ref_grad)) and verts.shape == ref_verts.shape and \
            bool(np.array_equal(verts, ref_verts))
        ms = _time_replays(m, reps)
        results.append(dict(launch=cfg, ms=ms, identical=same))
        if log:
            log(f"[tune] {cfg} {ms:.3f} ms identical={same}")
        if not same:
            raise RuntimeError(f"mapping {cfg} changed the result")
    best = min(results, key=lambda r: r["ms"])
    m.set_launch(**best["launch"])
    m.capture()
    entry = dict(launch=best["launch"], ms=best["ms"], points=len(results),
                 when=time.strftime("%Y-%m-%d %H:%M:%S"))
    if use_cache:
        cache[key] = entry
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            json.dump(cache, open(path, "w"), indent=1)
        except OSError:
            pass
    return dict(entry, cached=False, results=results)
