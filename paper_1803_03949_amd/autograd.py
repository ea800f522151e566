"""Differentiable extraction: torch.autograd.Function wrappers around the
library's forward and backward kernels.

Vertex positions depend on the TSDF through the edge interpolation of the
marching cubes (Sec. V-C) and on the depth frame through the running
average of the fusion (Eq. 2).  The backward passes hold the mesh
connectivity, the block set, the pixel each voxel projected to and every
branch of the fusion fixed.
"""
from __future__ import annotations

import numpy as np
import torch

from .binding import Volume


class TSDFMesh(torch.autograd.Function):
    """verts, tris, keys = TSDFMesh.apply(tsdf, weight, coords, vol).

    tsdf, weight: (n, 512) FP32 device tensors of the blocks at `coords`
    ((n, 3) int32); `vol` is a Volume used as the workspace (reset first).
    Returns vertex positions (V, 3) metres (differentiable), triangles
    (F, 3) int32 and edge keys (V,) int64."""

    @staticmethod
    def forward(ctx, tsdf, weight, coords, vol: Volume):
        vol.reset()
        vol.import_blocks(coords, tsdf.detach().contiguous(), weight.detach().contiguous())
        vol.extract(scope_all=True)
        vol.gc()
        verts, tris, keys = vol.download()
        ctx.vol = vol
        ctx.save_for_backward(vol.lookup(coords))
        ctx.mark_non_differentiable(tris, keys)
        return verts, tris, keys

    @staticmethod
    def backward(ctx, gverts, gtris, gkeys):
        (rows,) = ctx.saved_tensors
        g = ctx.vol.extract_backward(gverts.contiguous())
        return g[rows.long()], None, None, None


class FusedMesh(torch.autograd.Function):
    """verts, tris, keys = FusedMesh.apply(depth, tsdf0, weight0, coords, vol,
    K, cam_to_world, min_depth, max_depth).

    The blocks at `coords` start from tsdf0/weight0, the depth frame is fused
    into the volume (which may allocate further blocks), and the whole volume
    is meshed.  Gradients flow to depth (H, W) and to tsdf0."""

    @staticmethod
    def forward(ctx, depth, tsdf0, weight0, coords, vol: Volume, K, cam_to_world,
                min_depth=0.0, max_depth=1e30):
        vol.reset()
        vol.import_blocks(coords, tsdf0.detach().contiguous(), weight0.detach().contiguous())
        d = depth.detach().contiguous()
        vol.integrate(d, K, np.asarray(cam_to_world, np.float32), min_depth, max_depth)
        vol.extract(scope_all=True)
        vol.gc()
        verts, tris, keys = vol.download()
        ctx.vol = vol
        ctx.save_for_backward(d, vol.lookup(coords))
        ctx.mark_non_differentiable(tris, keys)
        return verts, tris, keys

    @staticmethod
    def backward(ctx, gverts, gtris, gkeys):
        depth, rows = ctx.saved_tensors
        g1 = ctx.vol.extract_backward(gverts.contiguous())
        g0, gD = ctx.vol.integrate_backward(depth, g1)
        return gD, g0[rows.long()], None, None, None, None, None, None, None
