"""ctypes binding of the voxmesh C-ABI (include/voxmesh.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream, every step of the method runs in the library's HIP kernels.  The
library is loaded from this package directory; if it is missing, or no GPU
is visible, the calls raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

# The library built in this package directory; VOXMESH_LIBRARY names another
# build of the same sources (e.g. to compare two builds side by side).
LIB_PATH = os.environ.get("VOXMESH_LIBRARY") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libvoxmesh.so")

VM_OK = 0
VM_SCOPE_DIRTY, VM_SCOPE_ALL = 0, 1
VM_EXTRACT_REFINE = 0x100
ERRORS = {
    -1: "VM_ERR_ARG", -2: "VM_ERR_HASH_FULL", -3: "VM_ERR_BLOCK_POOL_FULL",
    -4: "VM_ERR_VERTEX_POOL_FULL", -6: "VM_ERR_CAPACITY",
    -7: "VM_ERR_HIP", -8: "VM_ERR_RANGE",
}


class VmError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {ERRORS.get(code, code)}")


class vm_config(ctypes.Structure):
    _fields_ = [("voxel_m", ctypes.c_float), ("trunc_vox", ctypes.c_float),
                ("refine_eps_vox", ctypes.c_float), ("hash_log2", ctypes.c_int32),
                ("max_blocks", ctypes.c_int32), ("max_vertices", ctypes.c_int32),
                ("hash_mode", ctypes.c_int32),
                ("batch_volumes", ctypes.c_int32)]


class vm_launch(ctypes.Structure):
    _fields_ = [("wave_group_size", ctypes.c_int32), ("wave_groups_per_cu", ctypes.c_int32),
                ("block_groups_per_cu", ctypes.c_int32), ("item_groups_per_cu", ctypes.c_int32),
                ("block_order", ctypes.c_int32)]


LAUNCH_FIELDS = [f for f, _ in vm_launch._fields_]
SLOT_SPAN = 64  # stored block x of slot k, local x: 64k - 8192 + x
NOALLOC_MAX_BYTES = 64 << 20  # VM_NOALLOC_MAX_BYTES


class vm_batch_io(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_void_p), ("coords", ctypes.c_void_p),
                ("tsdf", ctypes.c_void_p), ("weight", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("rows", ctypes.c_void_p), ("pos", ctypes.c_void_p), ("slot_of", ctypes.c_void_p),
                ("pos_cap", ctypes.c_int64), ("dL_dpos", ctypes.c_void_p),
                ("dL_dtsdf", ctypes.c_void_p)]


VM_BATCH_FORWARD, VM_BATCH_BACKWARD = 1, 2


class vm_intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("min_depth_m", ctypes.c_float), ("max_depth_m", ctypes.c_float)]


_STATUS_FIELDS = ["blocks", "frame_blocks", "pending_blocks", "dirty_blocks", "vertex_blocks",
                  "changed_cubes", "vertex_slots", "free_vertex_slots", "triangles",
                  "tri_cubes", "new_vertices", "updated_vertices", "freed_vertices",
                  "refined_cubes", "vertex_segments", "segment_capacity", "max_segment_live"]


TOTALS = ["frames", "frame_blocks", "dirty_blocks", "vertex_blocks", "new_vertices",
          "updated_vertices", "changed_cubes", "new_triangles", "freed_vertices",
          "refined_cubes", "dropped_triangles", "moved_vertices"]
KERNELS = ["collect", "assign", "fuse", "import", "dirty", "classify", "refine", "vertices",
           "download", "backward", "counters", "ablation", "positions"]


class vm_status(ctypes.Structure):
    _fields_ = [("error", ctypes.c_int32), ("error_bits", ctypes.c_uint32)] + \
               [(n, ctypes.c_int64) for n in _STATUS_FIELDS]


_lib = None


def lib() -> ctypes.CDLL:
    """Load the HIP library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"voxmesh HIP library not built: {LIB_PATH} "
                               "(run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, I64 = ctypes.c_void_p, ctypes.c_int64
        PI64 = ctypes.POINTER(ctypes.c_int64)
        sigs = {
            "vm_volume_bytes": [ctypes.POINTER(vm_config), ctypes.POINTER(ctypes.c_size_t)],
            "vm_create_volume": [ctypes.POINTER(vm_config), P, ctypes.c_size_t, P,
                                 ctypes.POINTER(ctypes.c_void_p)],
            "vm_create_volume_noalloc": [ctypes.POINTER(vm_config), P,
                                         ctypes.POINTER(ctypes.c_void_p)],
            "vm_destroy_volume": [P],
            "vm_reset_volume": [P, P],
            "vm_integrate_depth": [P, P, ctypes.POINTER(vm_intrinsics), P, P],
            "vm_import_blocks": [P, P, P, P, I64, P],
            "vm_extract_mesh": [P, ctypes.c_int, P],
            "vm_refine_mesh": [P, P],
            "vm_gc": [P, P],
            "vm_download_mesh": [P, P, P, P, I64, I64, PI64, PI64, P],
            "vm_download_normals": [P, P, I64, P],
            "vm_download_births": [P, P, I64, P],
            "vm_sharing_ablation": [P, ctypes.c_int, P, P, P, P],
            "vm_bind_tsdf": [P, P, P],
            "vm_extract_backward": [P, P, P, P],
            "vm_integrate_backward": [P, P, P, P, P, P],
            "vm_get_status": [P, ctypes.POINTER(vm_status), P],
            "vm_export_blocks": [P, P, P, P, P, P, I64, PI64, P],
            "vm_export_vertices": [P, P, P, P, I64, PI64, P],
            "vm_export_block_list": [P, ctypes.c_int, P, I64, PI64, P],
            "vm_get_totals": [P, P, ctypes.c_int, P],
            "vm_lookup_blocks": [P, P, P, I64, P],
            "vm_import_batch": [P, P, P, P, P, I64, P, P],
            "vm_export_positions": [P, P, P, I64, P],
            "vm_extract_backward_slots": [P, P, P, I64, P, P],
            "vm_extract_batch": [P, ctypes.POINTER(vm_batch_io), ctypes.c_int, P],
            "vm_set_launch": [P, ctypes.POINTER(vm_launch)],
            "vm_get_launch": [P, ctypes.POINTER(vm_launch)],
            "vm_profile": [P, ctypes.c_int],
            "vm_profile_mask": [P, ctypes.c_uint32],
            "vm_profile_read": [P, P, P],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code: int, where: str, allow=()):
    if code != VM_OK and code not in allow:
        raise VmError(code, where)
    return code


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Volume:
    """One hashed TSDF volume with its mesh, in a torch-owned device buffer."""

    def __init__(self, voxel_m: float, trunc_vox: float = 4.0, refine_eps_vox: float = 0.5,
                 hash_log2: int = 20, max_blocks: int = 1 << 16, max_vertices: int = 1 << 22,
                 hash_mode: int = 0, batch_volumes: int = 0,
                 device=None, noalloc: bool = False):
        """noalloc: the workspace is the library's static per-device array
        (vm_create_volume_noalloc, at most NOALLOC_MAX_BYTES, one such
        volume per device at a time) instead of a torch buffer."""
        if not torch.cuda.is_available():
            raise RuntimeError("voxmesh needs a ROCm GPU (torch.cuda.is_available() is False)")
        L = lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.cfg = vm_config(voxel_m, trunc_vox, refine_eps_vox, hash_log2, max_blocks,
                             max_vertices, hash_mode, batch_volumes)
        nbytes = ctypes.c_size_t()
        _check(L.vm_volume_bytes(ctypes.byref(self.cfg), ctypes.byref(nbytes)), "vm_volume_bytes")
        self.nbytes = nbytes.value
        with torch.cuda.device(self.device):
            h = ctypes.c_void_p()
            if noalloc:
                self.mem = None
                _check(L.vm_create_volume_noalloc(ctypes.byref(self.cfg), _stream(),
                                                  ctypes.byref(h)), "vm_create_volume_noalloc")
            else:
                self.mem = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
                off = (-self.mem.data_ptr()) % 256
                self._base = self.mem.data_ptr() + off
                _check(L.vm_create_volume(ctypes.byref(self.cfg), self._base, self.nbytes,
                                          _stream(), ctypes.byref(h)), "vm_create_volume")
        self.h = h

    def close(self):
        """Release the handle now (a noalloc volume frees its device's
        static workspace for the next one)."""
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.vm_destroy_volume(h)
        self.h = None

    def __del__(self):
        self.close()

    # -- method steps ---------------------------------------------------------
    def integrate(self, depth: torch.Tensor, K, cam_to_world, min_depth=0.0, max_depth=1e30,
                  stream=None):
        assert depth.is_cuda and depth.dtype == torch.float32 and depth.is_contiguous()
        H, W = depth.shape
        fx, fy, cx, cy = K
        intr = vm_intrinsics(fx, fy, cx, cy, W, H, min_depth, max_depth)
        T = np.ascontiguousarray(cam_to_world, dtype=np.float32).reshape(16)
        _check(lib().vm_integrate_depth(self.h, _ptr(depth), ctypes.byref(intr), _ptr(T),
                                        _stream(stream)), "vm_integrate_depth")

    def import_blocks(self, coords: torch.Tensor, tsdf: torch.Tensor, weight: torch.Tensor,
                      stream=None):
        n = coords.shape[0]
        assert coords.is_cuda and coords.dtype == torch.int32 and coords.is_contiguous()
        assert tsdf.dtype == torch.float32 and weight.dtype == torch.float32
        assert tsdf.numel() >= 512 * n and weight.numel() >= 512 * n  # rows 0..n-1 are read
        _check(lib().vm_import_blocks(self.h, _ptr(coords), _ptr(tsdf), _ptr(weight), n,
                                      _stream(stream)), "vm_import_blocks")

    def bind_tsdf(self, tsdf: torch.Tensor | None, weight: torch.Tensor | None):
        """Use (max_blocks, 512) FP32 device tensors as the volume's TSDF and
        weight storage (imports then pass these same tensors and copy
        nothing); None, None returns to the volume's own arrays."""
        if tsdf is None and weight is None:
            _check(lib().vm_bind_tsdf(self.h, None, None), "vm_bind_tsdf")
            self._bound = None
            return
        B = self.cfg.max_blocks
        for t in (tsdf, weight):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
            assert t.numel() == 512 * B
        _check(lib().vm_bind_tsdf(self.h, _ptr(tsdf), _ptr(weight)), "vm_bind_tsdf")
        self._bound = (tsdf, weight)  # kept alive while bound

    def import_batch(self, slots: torch.Tensor | None, coords: torch.Tensor, tsdf: torch.Tensor,
                     weight: torch.Tensor, rows: torch.Tensor | None = None, stream=None):
        """Import blocks into slots of a batch (slots None for a plain volume);
        rows, if given ((n,) int32 device), receives each block's pool row."""
        n = coords.shape[0]
        assert coords.is_cuda and coords.dtype == torch.int32 and coords.is_contiguous()
        assert tsdf.dtype == torch.float32 and weight.dtype == torch.float32
        assert tsdf.numel() >= 512 * n and weight.numel() >= 512 * n  # rows 0..n-1 are read
        if slots is not None:
            assert slots.is_cuda and slots.dtype == torch.int32 and slots.numel() == n
        if rows is not None:
            assert rows.is_cuda and rows.dtype == torch.int32 and rows.numel() == n
        _check(lib().vm_import_batch(self.h, _ptr(slots), _ptr(coords), _ptr(tsdf), _ptr(weight),
                                     n, _ptr(rows), _stream(stream)), "vm_import_batch")

    def extract(self, scope_all: bool = False, stream=None, refine: bool = False):
        """Mesh extraction (dirty blocks, or every block with scope_all); with
        refine, each new type is refined (Eqs. 3-5) before it is meshed."""
        scope = (VM_SCOPE_ALL if scope_all else VM_SCOPE_DIRTY) | (VM_EXTRACT_REFINE if refine else 0)
        _check(lib().vm_extract_mesh(self.h, scope, _stream(stream)), "vm_extract_mesh")

    def refine(self, stream=None):
        _check(lib().vm_refine_mesh(self.h, _stream(stream)), "vm_refine_mesh")

    def gc(self, stream=None):
        _check(lib().vm_gc(self.h, _stream(stream)), "vm_gc")

    def reset(self, stream=None):
        _check(lib().vm_reset_volume(self.h, _stream(stream)), "vm_reset_volume")

    # -- results --------------------------------------------------------------
    def status(self, stream=None, check: bool = True) -> dict:
        st = vm_status()
        r = lib().vm_get_status(self.h, ctypes.byref(st), _stream(stream))
        out = {n: getattr(st, n) for n in ["error", "error_bits"] + _STATUS_FIELDS}
        if check:
            _check(r, "vm_get_status")
        return out

    def download(self, with_keys: bool = True, stream=None):
        """(verts (V,3) f32 metres, tris (F,3) i32, keys (V,) int64 or None)."""
        st = self.status(stream)
        vcap = max(1, st["vertex_slots"])
        tcap = max(1, st["triangles"])
        verts = torch.empty((vcap, 3), dtype=torch.float32, device=self.device)
        tris = torch.empty((tcap, 3), dtype=torch.int32, device=self.device)
        keys = torch.empty(vcap, dtype=torch.int64, device=self.device) if with_keys else None
        nv, nt = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().vm_download_mesh(self.h, _ptr(verts), _ptr(keys), _ptr(tris), vcap, tcap,
                                      ctypes.byref(nv), ctypes.byref(nt), _stream(stream)),
               "vm_download_mesh")
        verts, tris = verts[: nv.value], tris[: nt.value]
        self._dl_nv = nv.value
        return verts, tris, (keys[: nv.value] if keys is not None else None)

    def download_normals(self, stream=None) -> torch.Tensor:
        """Unit normals (V, 3) f32 of the vertices of the last download, in its
        row order (call right after `download`, before the volume changes)."""
        nv = getattr(self, "_dl_nv", 0)
        out = torch.empty((max(nv, 1), 3), dtype=torch.float32, device=self.device)
        _check(lib().vm_download_normals(self.h, _ptr(out), max(nv, 1), _stream(stream)),
               "vm_download_normals")
        return out[:nv]

    def sharing_ablation(self, scheme: int, edge_slot: torch.Tensor, edge_t: torch.Tensor,
                         counter: torch.Tensor, stream=None):
        """The paper's vertex-sharing schemes over the last extraction's dirty
        cubes (0: lock-based, 1: lock-free in four groups), on caller state:
        edge_slot int32 and edge_t float32 of max_blocks*3*512 entries
        (edge_slot -1 where no vertex), counter int32 (1,)."""
        _check(lib().vm_sharing_ablation(self.h, int(scheme), _ptr(edge_slot), _ptr(edge_t),
                                         _ptr(counter), _stream(stream)), "vm_sharing_ablation")

    def download_births(self, stream=None) -> torch.Tensor:
        """Birth frames (V,) int32 of the vertices of the last download, in its
        row order: the frame of the pass in which each vertex's count last
        became positive (frames count integrations and imports from 1)."""
        nv = getattr(self, "_dl_nv", 0)
        out = torch.empty(max(nv, 1), dtype=torch.int32, device=self.device)
        _check(lib().vm_download_births(self.h, _ptr(out), max(nv, 1), _stream(stream)),
               "vm_download_births")
        return out[:nv]

    def export_blocks(self, stream=None):
        n = ctypes.c_int64()
        _check(lib().vm_export_blocks(self.h, None, None, None, None, None, 0, ctypes.byref(n),
                                      _stream(stream)), "vm_export_blocks")
        m = n.value
        coords = np.zeros((max(m, 1), 3), np.int32)
        d = torch.empty((max(m, 1), 512), dtype=torch.float32, device=self.device)
        w = torch.empty_like(d)
        tp = torch.empty((max(m, 1), 512), dtype=torch.uint8, device=self.device)
        tc = torch.empty_like(tp)
        _check(lib().vm_export_blocks(self.h, _ptr(coords), _ptr(d), _ptr(w), _ptr(tp), _ptr(tc),
                                      m, ctypes.byref(n), _stream(stream)), "vm_export_blocks")
        return dict(coords=coords[:m], d=d[:m], w=w[:m], prev=tp[:m], cur=tc[:m])

    def export_vertices(self, stream=None):
        """Raw vertex pool: keys (int64, -1 for free slots), t, refcount."""
        n = ctypes.c_int64()
        _check(lib().vm_export_vertices(self.h, None, None, None, 0, ctypes.byref(n),
                                        _stream(stream)), "vm_export_vertices")
        m = n.value
        keys = torch.empty(max(m, 1), dtype=torch.int64, device=self.device)
        t = torch.empty(max(m, 1), dtype=torch.float32, device=self.device)
        ref = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        _check(lib().vm_export_vertices(self.h, _ptr(keys), _ptr(t), _ptr(ref), m,
                                        ctypes.byref(n), _stream(stream)), "vm_export_vertices")
        return dict(keys=keys[:m], t=t[:m], ref=ref[:m])

    def block_list(self, which: str, stream=None) -> np.ndarray:
        code = {"frame": 0, "dirty": 1, "pending": 2}[which]
        n = ctypes.c_int64()
        _check(lib().vm_export_block_list(self.h, code, None, 0, ctypes.byref(n), _stream(stream)),
               "vm_export_block_list")
        out = np.zeros((max(n.value, 1), 3), np.int32)
        _check(lib().vm_export_block_list(self.h, code, _ptr(out), n.value, ctypes.byref(n),
                                          _stream(stream)), "vm_export_block_list")
        return out[: n.value]

    def lookup(self, coords: torch.Tensor, stream=None) -> torch.Tensor:
        """Pool rows of the blocks at `coords` (device (n,3) int32), -1 if absent."""
        assert coords.is_cuda and coords.dtype == torch.int32 and coords.is_contiguous()
        out = torch.empty(coords.shape[0], dtype=torch.int32, device=self.device)
        _check(lib().vm_lookup_blocks(self.h, _ptr(coords), _ptr(out), coords.shape[0],
                                      _stream(stream)), "vm_lookup_blocks")
        return out

    # -- measurement ------------------------------------------------------------
    def totals(self, stream=None) -> dict:
        out = np.zeros(len(TOTALS), np.int64)
        _check(lib().vm_get_totals(self.h, _ptr(out), len(TOTALS), _stream(stream)), "vm_get_totals")
        return dict(zip(TOTALS, (int(x) for x in out)))

    def profile(self, enable: bool, kernels=None):
        """Time kernel launches (each launch records its start and end in two
        events): all kernels, or only those named in `kernels` (names as in
        KERNELS)."""
        if kernels is None or not enable:
            _check(lib().vm_profile(self.h, 1 if enable else 0), "vm_profile")
        else:
            mask = 0
            for k in kernels:
                mask |= 1 << KERNELS.index(k)
            _check(lib().vm_profile_mask(self.h, mask), "vm_profile_mask")

    def profile_read(self) -> dict:
        """{kernel: (launches, total ms)} of the recorded launches."""
        n = np.zeros(len(KERNELS), np.int64)
        ms = np.zeros(len(KERNELS), np.float64)
        _check(lib().vm_profile_read(self.h, _ptr(n), _ptr(ms)), "vm_profile_read")
        return {k: (int(a), float(b)) for k, a, b in zip(KERNELS, n, ms) if a}

    # -- gradients -------------------------------------------------------------
    def extract_backward(self, dL_dverts: torch.Tensor, out: torch.Tensor | None = None,
                         stream=None) -> torch.Tensor:
        """dL/d(fused TSDF) in block pool order, (blocks, 512)."""
        nb = self.status(stream)["blocks"]
        if out is None:
            out = torch.empty((max(nb, 1), 512), dtype=torch.float32, device=self.device)
        dL = dL_dverts.contiguous()
        _check(lib().vm_extract_backward(self.h, _ptr(dL), _ptr(out), _stream(stream)),
               "vm_extract_backward")
        return out[:nb]

    def positions(self, pos: torch.Tensor | None = None, slot_of: torch.Tensor | None = None,
                  stream=None):
        """Every vertex pool entry's position ((max_vertices, 3) metres, slot
        frame) and slot ((max_vertices,) int32, -1 without a live vertex);
        no synchronisation."""
        V = self.cfg.max_vertices
        if pos is None:
            pos = torch.empty((V, 3), dtype=torch.float32, device=self.device)
        if slot_of is None:
            slot_of = torch.empty(V, dtype=torch.int32, device=self.device)
        _check(lib().vm_export_positions(self.h, _ptr(pos), _ptr(slot_of), pos.shape[0],
                                         _stream(stream)), "vm_export_positions")
        return pos, slot_of

    def extract_backward_slots(self, dL_dpos: torch.Tensor, rows: torch.Tensor | None,
                               out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """dL/d(TSDF) from per-pool-entry vertex gradients, for the blocks at
        pool rows `rows` ((n,) int32 device) in that order."""
        assert dL_dpos.is_contiguous() and dL_dpos.shape[0] >= self.cfg.max_vertices
        if rows is None:
            nb = self.status(stream)["blocks"]
            n = nb
        else:
            n = rows.shape[0]
        if out is None:
            out = torch.empty((max(n, 1), 512), dtype=torch.float32, device=self.device)
        _check(lib().vm_extract_backward_slots(self.h, _ptr(dL_dpos), _ptr(rows), n, _ptr(out),
                                               _stream(stream)), "vm_extract_backward_slots")
        return out[:n]

    def batch_io(self, slots, coords, tsdf, weight, rows, pos, slot_of, dL_dpos, dL_dtsdf):
        """vm_batch_io over device tensors (which the caller keeps alive and in
        place while graphs captured with it are replayed)."""
        n = coords.shape[0]
        for t, dt in ((coords, torch.int32), (tsdf, torch.float32), (weight, torch.float32),
                      (rows, torch.int32), (pos, torch.float32), (dL_dpos, torch.float32),
                      (dL_dtsdf, torch.float32)):
            assert t.is_cuda and t.dtype == dt and t.is_contiguous()
        assert tsdf.numel() >= 512 * n and weight.numel() >= 512 * n and rows.numel() == n
        assert dL_dtsdf.numel() >= 512 * n and dL_dpos.shape[0] >= pos.shape[0]
        if slots is not None:
            assert slots.is_cuda and slots.dtype == torch.int32 and slots.numel() == n
        if slot_of is not None:
            assert slot_of.is_cuda and slot_of.dtype == torch.int32 and slot_of.numel() >= pos.shape[0]
        return vm_batch_io(_ptr(slots), _ptr(coords), _ptr(tsdf), _ptr(weight), n, _ptr(rows),
                           _ptr(pos), _ptr(slot_of), pos.shape[0], _ptr(dL_dpos), _ptr(dL_dtsdf))

    def extract_batch(self, io: vm_batch_io, phase: int, stream=None):
        """vm_extract_batch: VM_BATCH_FORWARD or VM_BATCH_BACKWARD, each a
        graph the library captures once and replays (plain launches on a
        stream under capture or on the legacy default stream)."""
        _check(lib().vm_extract_batch(self.h, ctypes.byref(io), int(phase), _stream(stream)),
               "vm_extract_batch")

    def set_launch(self, **kw):
        cur = self.get_launch()
        cur.update(kw)
        l = vm_launch(*(int(cur[f]) for f in LAUNCH_FIELDS))
        _check(lib().vm_set_launch(self.h, ctypes.byref(l)), "vm_set_launch")

    def get_launch(self) -> dict:
        l = vm_launch()
        _check(lib().vm_get_launch(self.h, ctypes.byref(l)), "vm_get_launch")
        return {f: int(getattr(l, f)) for f in LAUNCH_FIELDS}

    def integrate_backward(self, depth: torch.Tensor, dL_dtsdf1: torch.Tensor, stream=None):
        """(dL/d(TSDF before the last fusion), dL/d(depth)) for the last frame."""
        g1 = dL_dtsdf1.contiguous()
        g0 = torch.empty_like(g1)
        gD = torch.empty_like(depth)
        _check(lib().vm_integrate_backward(self.h, _ptr(depth), _ptr(g1), _ptr(g0), _ptr(gD),
                                           _stream(stream)), "vm_integrate_backward")
        return g0, gD


def key_to_edge(keys) -> np.ndarray:
    """Edge keys -> (n, 4) int (gx, gy, gz, axis)."""
    k = np.asarray(keys.cpu() if isinstance(keys, torch.Tensor) else keys).astype(np.int64)
    axis = k & 3
    local = (k >> 2) & 511
    bz = ((k >> 11) & 0x3FFF) - 8192
    by = ((k >> 25) & 0x3FFF) - 8192
    bx = ((k >> 39) & 0x3FFF) - 8192
    return np.stack([8 * bx + (local & 7), 8 * by + ((local >> 3) & 7), 8 * bz + (local >> 6),
                     axis], axis=1)
