"""Stage II of Alg.1 (Sec. 4.2): adaptive assignment of occupied voxels to
local fields, and the uniform block decomposition (360Roam-u, Sec. 6).

Both run in the library's HIP kernels (r360_assign_fields,
r360_assign_uniform); this module only marshals arguments. The returned
field map (int32 [n2, n1, n0], -1 where unoccupied) goes straight into
Scene(occ, field_map, ...).
"""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import check, lib
from .render import _dev, _ptr, _stream


def _dims(occ: torch.Tensor):
    if occ.dim() != 3:
        raise ValueError("occ must be [n2, n1, n0]")
    return (C.c_int32 * 3)(occ.shape[2], occ.shape[1], occ.shape[0])


def assign_fields(occ: torch.Tensor, threshold: float, n_fields: int):
    """(field_map, S): n_fields fields of floor(S/n) or ceil(S/n) occupied voxels each."""
    occ = _dev(occ, torch.float32, "occ")
    n = _dims(occ)
    need = int(lib().r360_assign_workspace_bytes(n))
    if need == 0:
        raise ValueError(f"invalid grid: {lib().r360_last_error().decode()}")
    ws = torch.empty(need, dtype=torch.uint8, device=occ.device)
    fmap = torch.empty(occ.shape, dtype=torch.int32, device=occ.device)
    S = C.c_int64(0)
    check(lib().r360_assign_fields(n, _ptr(occ), threshold, n_fields, _ptr(fmap), C.byref(S), _ptr(ws), ws.numel(),
                                   _stream()))
    return fmap, int(S.value)


def assign_uniform(occ: torch.Tensor, threshold: float, blocks):
    """(field_map, n_fields) for blocks = (b0, b1, b2) equal blocks per axis."""
    occ = _dev(occ, torch.float32, "occ")
    n = _dims(occ)
    b = (C.c_int32 * 3)(*[int(x) for x in blocks])
    need = int(lib().r360_assign_uniform_workspace_bytes(b))
    if need == 0:
        raise ValueError("invalid block counts")
    ws = torch.empty(need, dtype=torch.uint8, device=occ.device)
    fmap = torch.empty(occ.shape, dtype=torch.int32, device=occ.device)
    nf = C.c_int32(0)
    check(lib().r360_assign_uniform(n, _ptr(occ), threshold, b, _ptr(fmap), C.byref(nf), _ptr(ws), ws.numel(),
                                    _stream()))
    return fmap, int(nf.value)
