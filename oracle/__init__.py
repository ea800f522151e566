"""CPU oracle for the incremental volumetric mesh (Dong et al., arXiv 1803.03949).

TEST INFRASTRUCTURE ONLY.  The tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` are the only callers.  The product library never
imports this package and shares no code with it.

``oracle.cpp`` is a scalar, single-threaded C++17 implementation of the
paper's steps (Eq. 1 block collection, Eq. 2 fusion, Sec. V-B..V-E meshing,
Eqs. 3-5 refinement) plus an FP64 twin for gradients.  This module compiles it
with g++ and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (no contraction, no fast-math, exact IEEE FP32)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-fPIC", "-shared", "-o", tmp, _SRC,
        ])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        vp, i, f, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double
        P = ctypes.c_void_p
        sig = {
            "orc_create": (vp, [f, f, f]),
            "orc_destroy": (None, [vp]),
            "orc_set_threads": (None, [vp, i]),
            "orc_keep_fusion": (None, [vp, i]),
            "orc_integrate": (i, [vp, P, i, i, f, f, f, f, f, f, P]),
            "orc_restrict_blocks": (None, [vp, P, i]),
            "orc_import_blocks": (i, [vp, P, P, P, i]),
            "orc_extract": (i, [vp, i]),
            "orc_extract_refine": (i, [vp, i]),
            "orc_refine": (i, [vp]),
            "orc_gc": (i, [vp]),
            "orc_num_blocks": (i, [vp]),
            "orc_export_blocks": (None, [vp, P, P, P, P, P]),
            "orc_num_set": (i, [vp, i]),
            "orc_export_set": (None, [vp, i, P]),
            "orc_num_vertices": (i, [vp, i]),
            "orc_export_vertices": (None, [vp, i, P, P, P]),
            "orc_num_triangles": (i, [vp]),
            "orc_export_triangles": (None, [vp, P]),
            "orc_download": (None, [vp, P, P]),
            "orc_cube_triangles": (i, [i, P]),
            "orc_cube_polygon_sizes": (i, [i, P]),
            "orc_cube_polygons": (i, [i, P, P]),
            "orc_refine_type": (i, [i, i, P, f]),
            "orc_regular_type": (i, [i]),
            "orc_corner_offsets": (None, [P]),
            "orc_edge_ends": (None, [P]),
            "orc_grad_tsdf64": (None, [vp, P, P]),
            "orc_positions64": (None, [vp, i, i, i, d, P]),
            "orc_normals64": (None, [vp, P, P]),
            "orc_export_births": (None, [vp, P]),
            "orc_grad_fusion64": (None, [vp, P, P, P]),
            "orc_positions64_depth": (None, [vp, i, d, P]),
            "orc_num_fused": (i, [vp]),
            "orc_export_fused": (None, [vp, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ----- table-level helpers ---------------------------------------------------

def cube_triangles(cube_type: int) -> np.ndarray:
    """Triangles of one cube type as (n, 3) cube-edge numbers."""
    out = np.zeros(15, np.int32)
    n = lib().orc_cube_triangles(int(cube_type), _ptr(out))
    if n < 0:
        raise RuntimeError(f"face segments of type {cube_type} do not close")
    return out[: 3 * n].reshape(n, 3).copy()


def cube_polygon_sizes(cube_type: int) -> list[int]:
    out = np.zeros(8, np.int32)
    n = lib().orc_cube_polygon_sizes(int(cube_type), _ptr(out))
    if n < 0:
        raise RuntimeError(f"face segments of type {cube_type} do not close")
    return [int(x) for x in out[:n]]


def cube_polygons(cube_type: int) -> list[list[int]]:
    """Closed polygons of one cube type as cyclic lists of cube-edge numbers."""
    sizes = np.zeros(8, np.int32)
    edges = np.zeros(12, np.int32)
    n = lib().orc_cube_polygons(int(cube_type), _ptr(sizes), _ptr(edges))
    if n < 0:
        raise RuntimeError(f"face segments of type {cube_type} do not close")
    out, k = [], 0
    for s in sizes[:n]:
        out.append([int(e) for e in edges[k:k + s]])
        k += s
    return out


def refine_type(t: int, prev: int, dcorner, eps: float) -> int:
    dc = np.ascontiguousarray(dcorner, dtype=np.float32)
    assert dc.shape == (8,)
    return lib().orc_refine_type(int(t), int(prev), _ptr(dc), float(eps))


def regular_types() -> list[int]:
    return [lib().orc_regular_type(j) for j in range(6)]


def corner_offsets() -> np.ndarray:
    out = np.zeros((8, 3), np.int32)
    lib().orc_corner_offsets(_ptr(out))
    return out


def edge_ends() -> np.ndarray:
    out = np.zeros((12, 2), np.int32)
    lib().orc_edge_ends(_ptr(out))
    return out


# ----- the volume -------------------------------------------------------------

class OracleVolume:
    """One hashed TSDF volume with its mesh, on the host."""

    def __init__(self, voxel_m: float, trunc_vox: float = 4.0, refine_eps_vox: float = 0.5,
                 threads: int = 1, keep_fusion: bool = True):
        """threads: threads of the loops over blocks (the result does not
        depend on it); keep_fusion: keep per-voxel records of the last
        fusion for grad_fusion64 (off for long forward-only sequences)."""
        self.voxel_m = float(np.float32(voxel_m))
        self._h = lib().orc_create(float(voxel_m), float(trunc_vox), float(refine_eps_vox))
        lib().orc_set_threads(self._h, int(threads))
        lib().orc_keep_fusion(self._h, 1 if keep_fusion else 0)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    # -- method steps --
    def integrate(self, depth: np.ndarray, K, cam_to_world: np.ndarray,
                  min_depth: float = 0.0, max_depth: float = 1e30) -> int:
        depth = np.ascontiguousarray(depth, dtype=np.float32)
        H, W = depth.shape
        T = np.ascontiguousarray(cam_to_world, dtype=np.float32).reshape(16)
        fx, fy, cx, cy = (float(np.float32(x)) for x in K)
        return lib().orc_integrate(self._h, _ptr(depth), W, H, fx, fy, cx, cy,
                                   float(min_depth), float(max_depth), _ptr(T))

    def restrict(self, coords) -> None:
        """Collect only these blocks in later integrations (None: all).  The
        collected blocks' TSDF and weights are exactly those of a full run."""
        c = np.ascontiguousarray(np.zeros((0, 3)) if coords is None else coords,
                                 dtype=np.int32).reshape(-1, 3)
        lib().orc_restrict_blocks(self._h, _ptr(c), c.shape[0])

    def import_blocks(self, coords: np.ndarray, d: np.ndarray, w: np.ndarray) -> int:
        coords = np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 3)
        n = coords.shape[0]
        d = np.ascontiguousarray(d, dtype=np.float32).reshape(n, 512)
        w = np.ascontiguousarray(w, dtype=np.float32).reshape(n, 512)
        r = lib().orc_import_blocks(self._h, _ptr(coords), _ptr(d), _ptr(w), n)
        if r < 0:
            raise ValueError("block coordinate out of range")
        return r

    def extract(self, scope_all: bool = False, refine: bool = False) -> int:
        """Sec. V-B..V-D; with refine, Eqs. 3-5 applied to each new type first (Sec. V-F)."""
        f = lib().orc_extract_refine if refine else lib().orc_extract
        return f(self._h, 1 if scope_all else 0)

    def refine(self) -> int:
        return lib().orc_refine(self._h)

    def gc(self) -> int:
        return lib().orc_gc(self._h)

    # -- inspection --
    def blocks(self):
        n = lib().orc_num_blocks(self._h)
        coords = np.zeros((n, 3), np.int32)
        d = np.zeros((n, 512), np.float32)
        w = np.zeros((n, 512), np.float32)
        prev = np.zeros((n, 512), np.uint8)
        cur = np.zeros((n, 512), np.uint8)
        lib().orc_export_blocks(self._h, _ptr(coords), _ptr(d), _ptr(w), _ptr(prev), _ptr(cur))
        return dict(coords=coords, d=d, w=w, prev=prev, cur=cur)

    def block_set(self, which: str) -> np.ndarray:
        code = {"frame": 0, "dirty": 1, "pending": 2}[which]
        n = lib().orc_num_set(self._h, code)
        out = np.zeros((n, 3), np.int32)
        lib().orc_export_set(self._h, code, _ptr(out))
        return out

    def vertices(self, live_only: bool = True):
        n = lib().orc_num_vertices(self._h, 1 if live_only else 0)
        keys = np.zeros((n, 4), np.int32)
        t = np.zeros(n, np.float32)
        ref = np.zeros(n, np.int32)
        lib().orc_export_vertices(self._h, 1 if live_only else 0, _ptr(keys), _ptr(t), _ptr(ref))
        return dict(keys=keys, t=t, ref=ref)

    def triangles(self) -> np.ndarray:
        """(F, 3, 4) edge keys (gx, gy, gz, axis) of every triangle."""
        n = lib().orc_num_triangles(self._h)
        keys = np.zeros((n, 3, 4), np.int32)
        lib().orc_export_triangles(self._h, _ptr(keys))
        return keys

    def download(self):
        nv = lib().orc_num_vertices(self._h, 1)
        nt = lib().orc_num_triangles(self._h)
        verts = np.zeros((nv, 3), np.float32)
        tris = np.zeros((nt, 3), np.int32)
        lib().orc_download(self._h, _ptr(verts), _ptr(tris))
        return verts, tris

    # -- FP64 gradients --
    def grad_tsdf64(self, dL_dv: np.ndarray) -> np.ndarray:
        n = lib().orc_num_blocks(self._h)
        dL_dv = np.ascontiguousarray(dL_dv, dtype=np.float64)
        out = np.zeros((n, 512), np.float64)
        lib().orc_grad_tsdf64(self._h, _ptr(dL_dv), _ptr(out))
        return out

    def births(self) -> np.ndarray:
        """Birth frame (n_live,) of each live vertex, key order: the frame of
        the pass at whose end its count last became positive."""
        n = lib().orc_num_vertices(self._h, 1)
        out = np.zeros(n, np.int32)
        lib().orc_export_births(self._h, _ptr(out))
        return out

    def normals64(self):
        """FP64 unit normals (n_live, 3) of the live vertices in key order, and
        the gradient length before normalisation (n_live,): the TSDF gradient
        (central differences over observed voxels, one-sided at the edge of
        the observed region) interpolated along the vertex's edge at t."""
        n = lib().orc_num_vertices(self._h, 1)
        out = np.zeros((n, 3), np.float64)
        ln = np.zeros(n, np.float64)
        lib().orc_normals64(self._h, _ptr(out), _ptr(ln))
        return out, ln

    def positions64(self, voxel=(0, 0, 0), delta: float = 0.0) -> np.ndarray:
        nv = lib().orc_num_vertices(self._h, 1)
        out = np.zeros((nv, 3), np.float64)
        gx, gy, gz = (int(x) for x in voxel)
        lib().orc_positions64(self._h, gx, gy, gz, float(delta), _ptr(out))
        return out

    def grad_fusion64(self, dL_dd1: np.ndarray, H: int, W: int):
        n = lib().orc_num_blocks(self._h)
        dL_dd1 = np.ascontiguousarray(dL_dd1, dtype=np.float64).reshape(n, 512)
        dd0 = np.zeros((n, 512), np.float64)
        dD = np.zeros((H, W), np.float64)
        lib().orc_grad_fusion64(self._h, _ptr(dL_dd1), _ptr(dd0), _ptr(dD))
        return dd0, dD

    def positions64_depth(self, pixel: int, delta: float) -> np.ndarray:
        nv = lib().orc_num_vertices(self._h, 1)
        out = np.zeros((nv, 3), np.float64)
        lib().orc_positions64_depth(self._h, int(pixel), float(delta), _ptr(out))
        return out

    def fused(self):
        n = lib().orc_num_fused(self._h)
        ints = np.zeros((n, 5), np.int32)
        vals = np.zeros((n, 2), np.float64)
        lib().orc_export_fused(self._h, _ptr(ints), _ptr(vals))
        return dict(voxel=ints[:, :3], pixel=ints[:, 3], clamped=ints[:, 4],
                    d0=vals[:, 0], w0=vals[:, 1])
