"""voxmesh: incremental mesh extraction over a spatially hashed TSDF on
MI355X (gfx950), after Dong et al., arXiv 1803.03949.

The method runs in the HIP library ``libvoxmesh.so`` behind the C-ABI of
``include/voxmesh.h``; ``binding`` wraps it with ctypes and torch tensors.
"""
from .binding import (VM_SCOPE_ALL, VM_SCOPE_DIRTY, Volume, VmError, key_to_edge, lib)

__all__ = ["Volume", "VmError", "key_to_edge", "lib", "VM_SCOPE_ALL", "VM_SCOPE_DIRTY"]
