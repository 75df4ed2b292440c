"""Distillation of the global field into the local fields (Sec. 4.2, Eq.7).

global_points() evaluates the global field at given points (the targets);
distill_step() runs the local fields' forward, the per-field averaged
squared error of Eq.7 and its backward. Both run in the library's HIP
kernels (r360_global_field_points, r360_distill_step); this module only
marshals arguments.
"""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import check, lib
from .render import GlobalField, Scene, _dev, _opts, _ptr, _stream


def global_points(field: GlobalField, weights: torch.Tensor, x: torch.Tensor, d: torch.Tensor):
    """(sigma [M], rgb [3, M]) of the global field at points x with view directions d ([3, M])."""
    weights = _dev(weights, torch.float32, "weights")
    x = _dev(x, torch.float32, "x"); d = _dev(d, torch.float32, "d")
    M = x.shape[1]
    need = int(lib().r360_global_points_workspace_bytes(C.byref(field.desc), M))
    if need == 0:
        raise ValueError("invalid global-field description or point count")
    ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    sigma = torch.empty(M, dtype=torch.float32, device=x.device)
    rgb = torch.empty(3, M, dtype=torch.float32, device=x.device)
    check(lib().r360_global_field_points(C.byref(field.desc), _ptr(weights), _ptr(x), _ptr(d), M, _ptr(sigma),
                                         _ptr(rgb), _ptr(ws), ws.numel(), _stream()))
    return sigma, rgb


def distill_step(scene: Scene, x: torch.Tensor, d: torch.Tensor, field: torch.Tensor, target_sigma: torch.Tensor,
                 target_rgb: torch.Tensor, *, precision="bf16", grad: torch.Tensor = None):
    """(loss [1], grad [n_fields, P]) of Eq.7 on the scene's current weights."""
    x = _dev(x, torch.float32, "x"); d = _dev(d, torch.float32, "d")
    field = _dev(field, torch.int32, "field")
    ts = _dev(target_sigma, torch.float32, "target_sigma"); tr = _dev(target_rgb, torch.float32, "target_rgb")
    M = x.shape[1]
    opts = _opts(scene, 0.0, 1.0, 1, precision)
    ws = scene.workspace(M, 1)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    if grad is None:
        grad = torch.empty(scene.n_fields, scene.P, dtype=torch.float32, device=x.device)
    check(lib().r360_distill_step(scene._h, _ptr(x), _ptr(d), _ptr(field), M, _ptr(ts), _ptr(tr), C.byref(opts),
                                  _ptr(loss), _ptr(grad), _ptr(ws), ws.numel(), _stream()))
    return loss, grad
