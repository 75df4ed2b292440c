"""Stage I of Alg.1 (Sec. 4.1): progressive probabilistic occupancy.

The global field measures each ray (depth over normalised Eq.5 weights, the
spread of those weights as uncertainty, and opacity); every sampling
position then updates a logit grid by Eq.6 (clamped to [-2, 3.5], occupied
above probability 0.97). Both steps run in the library's HIP kernels
(r360_global_field_measure / r360_depth_uncertainty and
r360_occupancy_update); this module only marshals arguments.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import torch

from . import _lib
from ._lib import check, lib
from .render import GlobalField, _dev, _ptr, _stream

P_OCCUPIED = 0.97          # Sec. 4.1: occupied above this probability
LOGIT_RANGE = (-2.0, 3.5)  # Sec. 4.1: probability 0.12 to 0.97


def depth_uncertainty(t: torch.Tensor, delta: torch.Tensor, sigma: torch.Tensor):
    """Per-ray (depth, uncertainty, opacity) from dense [N, S] samples."""
    t = _dev(t, torch.float32, "t"); delta = _dev(delta, torch.float32, "delta")
    sigma = _dev(sigma, torch.float32, "sigma")
    if t.dim() != 2 or t.shape != delta.shape or t.shape != sigma.shape:
        raise ValueError("t, delta and sigma must share one [N, S] shape")
    N, S = t.shape
    out = [torch.empty(N, dtype=torch.float32, device=t.device) for _ in range(3)]
    check(lib().r360_depth_uncertainty(_ptr(t), _ptr(delta), _ptr(sigma), N, S, *(_ptr(x) for x in out), _stream()))
    return tuple(out)


def global_measure(field: GlobalField, weights: torch.Tensor, o: torch.Tensor, d: torch.Tensor,
                   chunk: int = 16384):
    """The global field's per-ray (depth, uncertainty, opacity) over o, d [3, N],
    in chunks of `chunk` rays (the forward's workspace grows with the chunk)."""
    weights = _dev(weights, torch.float32, "weights")
    o = _dev(o, torch.float32, "o"); d = _dev(d, torch.float32, "d")
    N = o.shape[1]
    out = [torch.empty(N, dtype=torch.float32, device=o.device) for _ in range(3)]
    for b in range(0, N, chunk):
        n = min(chunk, N - b)
        ob, db = o[:, b:b + n].contiguous(), d[:, b:b + n].contiguous()
        ws = field.workspace(n, o.device)
        check(lib().r360_global_field_measure(C.byref(field.desc), _ptr(weights), _ptr(ob), _ptr(db), n,
                                              *(_ptr(x[b:b + n]) for x in out), _ptr(ws), ws.numel(), _stream()))
    return tuple(out)


class OccupancyMap:
    """FP32 logit grid [n2, n1, n0] over lo + [0, n * voxel) (x fastest),
    starting at 0 (probability 1/2), updated one sampling position at a time."""

    def __init__(self, n=128, lo=-4.0, voxel: float = 0.0625, *, near: float = 0.0, far: float = float("inf"),
                 p_hit: float = 0.7, p_miss: float = 0.4, l_min: float = LOGIT_RANGE[0],
                 l_max: float = LOGIT_RANGE[1], min_opacity: float = 0.5, device="cuda"):
        g = _lib.OccDesc()
        n0 = n[0] if isinstance(n, (tuple, list)) else n
        lo0 = lo[0] if isinstance(lo, (tuple, list)) else lo
        check(lib().r360_occ_desc_init(C.byref(g), n0, lo0, voxel, near, far, p_hit, p_miss, l_min, l_max,
                                       min_opacity))
        if isinstance(n, (tuple, list)):
            g.n[:] = list(n)
        if isinstance(lo, (tuple, list)):
            g.lo[:] = list(lo)
        need = int(lib().r360_occupancy_workspace_bytes(C.byref(g)))
        if need == 0:
            raise ValueError(f"invalid occupancy description: {lib().r360_last_error().decode()}")
        self.desc = g
        shape = (g.n[2], g.n[1], g.n[0])
        self.logit = torch.zeros(shape, dtype=torch.float32, device=device)
        self.prob = torch.full(shape, 0.5, dtype=torch.float32, device=device)
        self._ws = torch.empty(need, dtype=torch.uint8, device=device)

    def update(self, o: torch.Tensor, d: torch.Tensor, depth: torch.Tensor, uncert: torch.Tensor,
               opacity: torch.Tensor, prob: bool = True):
        """One sampling position's rays o, d [3, N] and measurements [N]."""
        o = _dev(o, torch.float32, "o"); d = _dev(d, torch.float32, "d")
        depth = _dev(depth, torch.float32, "depth"); uncert = _dev(uncert, torch.float32, "uncert")
        opacity = _dev(opacity, torch.float32, "opacity")
        N = o.shape[1]
        check(lib().r360_occupancy_update(C.byref(self.desc), _ptr(self.logit), _ptr(self.prob) if prob else None,
                                          _ptr(o), _ptr(d), N, _ptr(depth), _ptr(uncert), _ptr(opacity),
                                          _ptr(self._ws), self._ws.numel(), _stream()))

    def occupied(self) -> torch.Tensor:
        """Voxels whose probability exceeds 0.97 (from the last update's probabilities)."""
        return self.prob > P_OCCUPIED
