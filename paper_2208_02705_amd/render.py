"""Python face of the r360 hot path: scenes, renders, training steps.

Thin marshalling over the C ABI (``_lib``): tensors are passed by device
pointer on torch's current stream; all arithmetic runs in libr360's HIP
kernels. Every array here is a torch tensor on a ROCm device.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

L_XYZ, L_DIR = 10, 4


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return t.contiguous()


def field_params(hidden: int) -> int:
    return int(lib().r360_field_params(hidden, L_XYZ, L_DIR))


def precision_code(p) -> int:
    return _lib.PRECISIONS[p] if isinstance(p, str) else int(p)


def make_opts(near: float, far: float, max_samples: int, precision, samples_per_voxel: int = 1) -> _lib.RenderOpts:
    o = _lib.RenderOpts()
    o.near_, o.far_, o.max_samples, o.precision = near, far, max_samples, precision_code(precision)
    o.samples_per_voxel = samples_per_voxel
    return o


class Scene:
    """Occupancy grid + voxel->field labels + packed per-field MLP weights.

    occ: float32 [n2, n1, n0] occupancy probability (x fastest); field_map:
    int32 same shape (-1 = none); weights: float32 [n_fields, P] canonical
    order. The grid spans lo + [0, n * voxel) on each axis.
    """

    def __init__(self, occ: torch.Tensor, field_map: torch.Tensor, weights: torch.Tensor, *, lo=(-4.0, -4.0, -4.0),
                 voxel: float = 0.25, threshold: float = 0.5, hidden: int = 32, center=(0.0, 0.0, 0.0),
                 half_extent: float = 4.0):
        occ = _dev(occ, torch.float32, "occ")
        field_map = _dev(field_map, torch.int32, "field_map")
        weights = _dev(weights, torch.float32, "weights")
        if occ.dim() != 3 or tuple(field_map.shape) != tuple(occ.shape):
            raise ValueError("occ and field_map must be [n2, n1, n0] of the same shape")
        n_fields = weights.shape[0]
        if weights.dim() != 2 or weights.shape[1] != field_params(hidden):
            raise ValueError(f"weights must be [n_fields, {field_params(hidden)}]")
        g = _lib.GridDesc()
        g.n[:] = [occ.shape[2], occ.shape[1], occ.shape[0]]
        g.lo[:] = list(lo) if isinstance(lo, Sequence) else [lo] * 3
        g.voxel, g.threshold = voxel, threshold
        m = _lib.MlpDesc()
        m.n_fields, m.hidden, m.L_xyz, m.L_dir = n_fields, hidden, L_XYZ, L_DIR
        m.center[:] = list(center)
        m.half_extent = half_extent
        h = C.c_void_p()
        check(lib().r360_scene_create(C.byref(g), _ptr(occ), _ptr(field_map), C.byref(m), _ptr(weights), _stream(),
                                      C.byref(h)))
        self._h = h
        self.grid, self.mlp = g, m
        self.n_fields, self.hidden, self.P = n_fields, hidden, weights.shape[1]
        self.device = occ.device
        self.samples_per_voxel = 1          # samples per occupied voxel segment (render options)
        self._ws: Optional[torch.Tensor] = None

    @classmethod
    def from_synth(cls, sc, device="cuda", weights: Optional[torch.Tensor] = None) -> "Scene":
        """Build from a synth.Scene description (host arrays)."""
        occ = torch.from_numpy(sc.occ).to(device)
        fm = torch.from_numpy(sc.field_map).to(device)
        w = torch.from_numpy(sc.weights).to(device) if weights is None else weights
        s = cls(occ, fm, w, lo=(sc.lo,) * 3, voxel=sc.voxel, threshold=sc.threshold, hidden=sc.hidden,
                center=sc.center, half_extent=sc.half_extent)
        s.near, s.far, s.max_samples = sc.near, sc.far, sc.max_samples
        s.samples_per_voxel = getattr(sc, "samples_per_voxel", 1)
        fr = getattr(sc, "frames", None)
        if fr is not None:
            fr = torch.from_numpy(np.ascontiguousarray(fr, dtype=np.float32)).to(device)
            s.set_frames(fr[:, :3].contiguous(), fr[:, 3].contiguous())
        torch.cuda.current_stream().synchronize()
        return s

    def set_frames(self, centers: Optional[torch.Tensor], half_extents: Optional[torch.Tensor] = None):
        """Per-field encoding frames (centers [F, 3], half_extents [F]); None
        restores the scene-wide frame."""
        if centers is None:
            check(lib().r360_scene_set_frames(self._h, None, None, _stream()))
            return
        centers = _dev(centers, torch.float32, "centers")
        half_extents = _dev(half_extents, torch.float32, "half_extents")
        check(lib().r360_scene_set_frames(self._h, _ptr(centers), _ptr(half_extents), _stream()))

    def set_weights(self, weights: torch.Tensor):
        check(lib().r360_scene_set_weights(self._h, _ptr(_dev(weights, torch.float32, "weights")), _stream()))

    def workspace(self, n_rays: int, max_samples: int) -> torch.Tensor:
        need = int(lib().r360_workspace_bytes(self._h, n_rays, max_samples))
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def close(self):
        if getattr(self, "_h", None):
            lib().r360_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Equirect:
    """Per-resolution sine/cosine tables of an equirect camera (Eq.2/Eq.3)."""

    def __init__(self, W: int, H: int):
        h = C.c_void_p()
        check(lib().r360_equirect_create(W, H, C.byref(h)))
        self._h, self.W, self.H = h, W, H

    def tables(self):
        import numpy as np
        sp = np.empty(self.W, np.float32); cp = np.empty(self.W, np.float32)
        st = np.empty(self.H, np.float32); ct = np.empty(self.H, np.float32)
        check(lib().r360_equirect_tables(self._h, sp.ctypes.data, cp.ctypes.data, st.ctypes.data, ct.ctypes.data))
        return sp, cp, st, ct

    def rays(self, c2w, pix: Optional[torch.Tensor] = None, device="cuda", eye: float = 0.0):
        """Rays [3, N] of the given pixels (all in raster order without a list);
        eye != 0: one eye of an omni-directional stereo pair (signed half eye distance)."""
        N = self.W * self.H if pix is None else pix.numel()
        if pix is not None:
            pix = _dev(pix, torch.int64, "pix")
        o = torch.empty(3, N, dtype=torch.float32, device=device)
        d = torch.empty(3, N, dtype=torch.float32, device=device)
        if eye:
            check(lib().r360_ods_rays(self._h, _lib.c2w_arg(c2w), eye, _ptr(pix), N, _ptr(o), _ptr(d), _stream()))
        else:
            check(lib().r360_equirect_rays(self._h, _lib.c2w_arg(c2w), _ptr(pix), N, _ptr(o), _ptr(d), _stream()))
        return o, d

    def close(self):
        if getattr(self, "_h", None):
            lib().r360_equirect_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def field_frames(field_map: torch.Tensor, n_fields: int, *, lo=(-4.0, -4.0, -4.0), voxel: float = 0.25):
    """(centers [F, 3], half_extents [F]): the box of each field's voxels."""
    field_map = _dev(field_map, torch.int32, "field_map")
    g = _lib.GridDesc()
    g.n[:] = [field_map.shape[2], field_map.shape[1], field_map.shape[0]]
    g.lo[:] = list(lo) if isinstance(lo, Sequence) else [lo] * 3
    g.voxel, g.threshold = voxel, 0.5
    ws = torch.empty(int(lib().r360_field_frames_workspace_bytes(n_fields)), dtype=torch.uint8,
                     device=field_map.device)
    centers = torch.empty(n_fields, 3, dtype=torch.float32, device=field_map.device)
    halves = torch.empty(n_fields, dtype=torch.float32, device=field_map.device)
    check(lib().r360_field_frames(C.byref(g), _ptr(field_map), n_fields, _ptr(centers), _ptr(halves), _ptr(ws),
                                  ws.numel(), _stream()))
    return centers, halves


def _opts(scene: Scene, near, far, max_samples, precision):
    return make_opts(scene.near if near is None else near, scene.far if far is None else far,
                     scene.max_samples if max_samples is None else max_samples, precision,
                     getattr(scene, "samples_per_voxel", 1))


def sample_rays(scene: Scene, o: torch.Tensor, d: torch.Tensor, *, near=None, far=None, max_samples=None,
                with_voxel: bool = True):
    """Occupied-voxel samples in ray-major order (dict of trimmed tensors)."""
    o = _dev(o, torch.float32, "o"); d = _dev(d, torch.float32, "d")
    N = o.shape[1]
    opts = _opts(scene, near, far, max_samples, "fp32")
    cap = N * opts.max_samples
    dev = o.device
    t_mid = torch.empty(cap, dtype=torch.float32, device=dev)
    delta = torch.empty(cap, dtype=torch.float32, device=dev)
    ray = torch.empty(cap, dtype=torch.int32, device=dev)
    field = torch.empty(cap, dtype=torch.int32, device=dev)
    voxel = torch.empty(cap, dtype=torch.int32, device=dev) if with_voxel else None
    off = torch.empty(N + 1, dtype=torch.int32, device=dev)
    ws = scene.workspace(N, opts.max_samples)
    total = C.c_int64()
    check(lib().r360_sample_rays(scene._h, _ptr(o), _ptr(d), N, C.byref(opts), C.byref(total), _ptr(t_mid),
                                 _ptr(delta), _ptr(ray), _ptr(field), _ptr(voxel), _ptr(off), _ptr(ws), ws.numel(),
                                 _stream()))
    S = total.value
    out = dict(offsets=off, t_mid=t_mid[:S], delta=delta[:S], ray_id=ray[:S], field=field[:S])
    if with_voxel:
        out["voxel"] = voxel[:S]
    return out


def render_rays(scene: Scene, o: torch.Tensor, d: torch.Tensor, *, precision="fp32", near=None, far=None,
                max_samples=None, ws: Optional[torch.Tensor] = None, term_eps: float = 0.0, term_after: int = 0):
    """(rgb [3, N], depth [N], opacity [N]) for caller rays o, d [3, N].
    term_eps > 0: early ray termination after term_after samples (rays whose
    transmittance there is below term_eps stop)."""
    o = _dev(o, torch.float32, "o"); d = _dev(d, torch.float32, "d")
    N = o.shape[1]
    opts = _opts(scene, near, far, max_samples, precision)
    opts.term_eps, opts.term_after = term_eps, term_after
    ws = scene.workspace(N, opts.max_samples) if ws is None else ws
    rgb = torch.empty(3, N, dtype=torch.float32, device=o.device)
    depth = torch.empty(N, dtype=torch.float32, device=o.device)
    opac = torch.empty(N, dtype=torch.float32, device=o.device)
    check(lib().r360_render_rays(scene._h, _ptr(o), _ptr(d), N, C.byref(opts), _ptr(rgb), _ptr(depth), _ptr(opac),
                                 _ptr(ws), ws.numel(), _stream()))
    return rgb, depth, opac


def render_rays_noalloc(scene: Scene, o: torch.Tensor, d: torch.Tensor, rgb: torch.Tensor, depth: torch.Tensor,
                        opacity: torch.Tensor, *, precision="fp32", near=None, far=None, max_samples=None):
    """render_rays into caller-owned outputs (rgb [3, N], depth [N], opacity
    [N], FP32 on the rays' device) with the library's own device scratch in
    place of a workspace: no device memory is allocated by this call."""
    o = _dev(o, torch.float32, "o"); d = _dev(d, torch.float32, "d")
    N = o.shape[1]
    for name, t, shape in (("rgb", rgb, (3, N)), ("depth", depth, (N,)), ("opacity", opacity, (N,))):
        if tuple(t.shape) != shape or t.dtype != torch.float32 or t.device != o.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 tensor of shape {shape} on {o.device}")
    opts = _opts(scene, near, far, max_samples, precision)
    check(lib().r360_render_rays_noalloc(scene._h, _ptr(o), _ptr(d), N, C.byref(opts), _ptr(rgb), _ptr(depth),
                                         _ptr(opacity), _stream()))
    return rgb, depth, opacity


class EquirectRenderer:
    """Renders W x H equirect views; owns the tables and output buffers."""

    def __init__(self, scene: Scene, W: int, H: int, *, precision="bf16", near=None, far=None, max_samples=None,
                 term_eps: float = 0.0, term_after: int = 0):
        self.scene, self.eq = scene, Equirect(W, H)
        self.opts = _opts(scene, near, far, max_samples, precision)
        self.opts.term_eps, self.opts.term_after = term_eps, term_after
        self.ws = scene.workspace(W * H, self.opts.max_samples)
        dev = scene.device
        self.rgb = torch.empty(3, H, W, dtype=torch.float32, device=dev)
        self.depth = torch.empty(H, W, dtype=torch.float32, device=dev)
        self.opacity = torch.empty(H, W, dtype=torch.float32, device=dev)

    def __call__(self, c2w, eye: float = 0.0):
        """One view; eye != 0 renders that eye of an omni-directional stereo pair."""
        if eye:
            check(lib().r360_render_ods(self.scene._h, self.eq._h, _lib.c2w_arg(c2w), eye, C.byref(self.opts),
                                        _ptr(self.rgb), _ptr(self.depth), _ptr(self.opacity), _ptr(self.ws),
                                        self.ws.numel(), _stream()))
        else:
            check(lib().r360_render_equirect(self.scene._h, self.eq._h, _lib.c2w_arg(c2w), C.byref(self.opts),
                                             _ptr(self.rgb), _ptr(self.depth), _ptr(self.opacity), _ptr(self.ws),
                                             self.ws.numel(), _stream()))
        return self.rgb, self.depth, self.opacity


def render_equirect(scene: Scene, W: int, H: int, c2w, **kw):
    r = EquirectRenderer(scene, W, H, **kw)
    rgb, depth, opac = r(c2w)
    return rgb.clone(), depth.clone(), opac.clone()


def render_stereo(scene: Scene, W: int, H: int, c2w, ipd: float = 0.064, **kw):
    """Omni-directional stereo pair ((rgb, depth, opacity) of the left eye,
    then of the right) with the eyes ipd apart (Sec. 5's stereoscopic mode)."""
    r = EquirectRenderer(scene, W, H, **kw)
    out = []
    for eye in (-0.5 * ipd, 0.5 * ipd):
        rgb, depth, opac = r(c2w, eye=eye)
        out.append((rgb.clone(), depth.clone(), opac.clone()))
    return tuple(out)


class PinholeRenderer:
    """Renders W x H perspective viewports (focal lengths fx, fy in pixels);
    owns the output buffers and shares the scene's workspace."""

    def __init__(self, scene: Scene, W: int, H: int, fx: float, fy: float, *, precision="bf16", near=None,
                 far=None, max_samples=None):
        self.scene, self.W, self.H, self.fx, self.fy = scene, W, H, fx, fy
        self.opts = _opts(scene, near, far, max_samples, precision)
        self.ws = scene.workspace(W * H, self.opts.max_samples)
        dev = scene.device
        self.rgb = torch.empty(3, H, W, dtype=torch.float32, device=dev)
        self.depth = torch.empty(H, W, dtype=torch.float32, device=dev)
        self.opacity = torch.empty(H, W, dtype=torch.float32, device=dev)

    def __call__(self, c2w):
        check(lib().r360_render_pinhole(self.scene._h, self.W, self.H, self.fx, self.fy, _lib.c2w_arg(c2w),
                                        C.byref(self.opts), _ptr(self.rgb), _ptr(self.depth), _ptr(self.opacity),
                                        _ptr(self.ws), self.ws.numel(), _stream()))
        return self.rgb, self.depth, self.opacity


def pinhole_rays(W: int, H: int, fx: float, fy: float, c2w, device="cuda"):
    """(o, d) [3, W*H] rays of a pinhole viewport, pixels in raster order."""
    o = torch.empty(3, W * H, dtype=torch.float32, device=device)
    d = torch.empty(3, W * H, dtype=torch.float32, device=device)
    check(lib().r360_pinhole_rays(W, H, fx, fy, _lib.c2w_arg(c2w), _ptr(o), _ptr(d), _stream()))
    return o, d


def render_pinhole(scene: Scene, W: int, H: int, fx: float, fy: float, c2w, **kw):
    r = PinholeRenderer(scene, W, H, fx, fy, **kw)
    return r(c2w)


def backward(scene: Scene, o, d, grad_rgb, *, precision="fp32", near=None, far=None, max_samples=None,
             ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Weight gradient [n_fields, P] of the most recent render_rays on `ws`."""
    o = _dev(o, torch.float32, "o"); d = _dev(d, torch.float32, "d")
    grad_rgb = _dev(grad_rgb, torch.float32, "grad_rgb")
    N = o.shape[1]
    opts = _opts(scene, near, far, max_samples, precision)
    ws = scene.workspace(N, opts.max_samples) if ws is None else ws
    g = torch.empty(scene.n_fields, scene.P, dtype=torch.float32, device=o.device)
    check(lib().r360_backward(scene._h, _ptr(o), _ptr(d), N, C.byref(opts), _ptr(grad_rgb), _ptr(g), _ptr(ws),
                              ws.numel(), _stream()))
    return g


def train_step(scene: Scene, o, d, target, *, precision="bf16", near=None, far=None, max_samples=None,
               grad: Optional[torch.Tensor] = None, loss: Optional[torch.Tensor] = None,
               rgb: Optional[torch.Tensor] = None):
    """Forward + L2 loss + backward: returns (loss [1], grad [n_fields, P])."""
    o = _dev(o, torch.float32, "o"); d = _dev(d, torch.float32, "d")
    target = _dev(target, torch.float32, "target")
    N = o.shape[1]
    opts = _opts(scene, near, far, max_samples, precision)
    ws = scene.workspace(N, opts.max_samples)
    dev = o.device
    grad = torch.empty(scene.n_fields, scene.P, dtype=torch.float32, device=dev) if grad is None else grad
    loss = torch.empty(1, dtype=torch.float32, device=dev) if loss is None else loss
    check(lib().r360_train_step(scene._h, _ptr(o), _ptr(d), N, _ptr(target), C.byref(opts), _ptr(loss), _ptr(grad),
                                _ptr(rgb), _ptr(ws), ws.numel(), _stream()))
    return loss, grad


def adam_step(w, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.99, eps: float = 1e-8):
    for t, n in ((w, "w"), (g, "g"), (m, "m"), (v, "v")):
        _dev(t, torch.float32, n)
    check(lib().r360_adam_step(_ptr(w), _ptr(g), _ptr(m), _ptr(v), w.numel(), step, lr, beta1, beta2, eps,
                               _stream()))


class GlobalField:
    """The global omnidirectional field stage (8 x width MLP with the encoding
    re-entering at the fifth layer) on BF16 MFMA GEMMs: forward, loss,
    backward and the per-cell density max into an occupancy grid."""

    def __init__(self, width: int = 256, color_width: int = 128, n_samples: int = 128, near: float = 0.1,
                 far: float = 20.0, center=(0.0, 0.0, 0.0), half_extent: float = 4.0, grid_n: int = 128,
                 grid_lo: float = -4.0, voxel: float = 0.0625):
        g = _lib.GlobalDesc()
        g.width, g.color_width, g.n_samples = width, color_width, n_samples
        g.near_, g.far_ = near, far
        g.center[:] = list(center)
        g.half_extent = half_extent
        g.grid_n[:] = [grid_n] * 3
        g.grid_lo[:] = [grid_lo] * 3
        g.voxel = voxel
        self.desc = g
        self.P = int(lib().r360_global_params(width, color_width))
        self._ws = None

    def workspace(self, n_rays: int, device) -> torch.Tensor:
        need = int(lib().r360_global_workspace_bytes(C.byref(self.desc), n_rays))
        if need == 0:
            raise ValueError("invalid global-field description")
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=device)
        return self._ws

    def step(self, weights: torch.Tensor, o: torch.Tensor, d: torch.Tensor, target: Optional[torch.Tensor] = None,
             occ: Optional[torch.Tensor] = None, grad: Optional[torch.Tensor] = None):
        """Returns dict(rgb [3, N], depth [N], loss [1] or None, grad [P] or None)."""
        weights = _dev(weights, torch.float32, "weights")
        o = _dev(o, torch.float32, "o"); d = _dev(d, torch.float32, "d")
        N = o.shape[1]
        dev = o.device
        ws = self.workspace(N, dev)
        rgb = torch.empty(3, N, dtype=torch.float32, device=dev)
        depth = torch.empty(N, dtype=torch.float32, device=dev)
        loss = None
        if target is not None:
            target = _dev(target, torch.float32, "target")
            loss = torch.empty(1, dtype=torch.float32, device=dev)
            grad = torch.empty(self.P, dtype=torch.float32, device=dev) if grad is None else grad
        else:
            grad = None
        if occ is not None:
            occ = _dev(occ, torch.float32, "occ")
        check(lib().r360_global_field_step(C.byref(self.desc), _ptr(weights), _ptr(o), _ptr(d), N, _ptr(target),
                                           _ptr(loss), _ptr(grad), _ptr(rgb), _ptr(depth), _ptr(occ), _ptr(ws),
                                           ws.numel(), _stream()))
        return dict(rgb=rgb, depth=depth, loss=loss, grad=grad)


def profile_enable(on: bool = True):
    """Per-stage HIP-event timing inside the library (see r360_profile_enable)."""
    check(lib().r360_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """{stage: (milliseconds, launches)} since the previous read."""
    ms = (C.c_double * _lib.NSTAGES)()
    cnt = (C.c_int32 * _lib.NSTAGES)()
    check(lib().r360_profile_read(ms, cnt))
    return {name: (ms[k], cnt[k]) for k, name in enumerate(_lib.STAGES)}


def lr_at(step: int, total: int, lr0: float = 1e-3, lr1: float = 5e-5) -> float:
    """Exponential decay from lr0 to lr1 over `total` steps (Sec. 6.3)."""
    lr = lib().r360_lr_schedule(step, total, lr0, lr1)
    if lr != lr:
        raise ValueError("lr0, lr1 must be positive and step >= 0")
    return lr


class RenderFunction(torch.autograd.Function):
    """rgb = render(weights; rays). Backward runs the hand-written compositing
    and MLP backward kernels; per-ray compositing is recomputed there."""

    @staticmethod
    def forward(ctx, weights, scene: Scene, o, d, precision="fp32", near=None, far=None, max_samples=None):
        scene.set_weights(weights.detach())
        opts = _opts(scene, near, far, max_samples, precision)
        ws = scene.workspace(o.shape[1], opts.max_samples)
        rgb, depth, opac = render_rays(scene, o, d, precision=precision, near=near, far=far,
                                       max_samples=max_samples, ws=ws)
        ctx.scene, ctx.kw = scene, dict(precision=precision, near=near, far=far, max_samples=max_samples)
        ctx.save_for_backward(o, d)
        ctx.ws = ws
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        o, d = ctx.saved_tensors
        g = backward(ctx.scene, o, d, grad_rgb.contiguous(), ws=ctx.ws, **ctx.kw)
        return g, None, None, None, None, None, None, None


class GradcheckFunction(torch.autograd.Function):
    """FP64 form of RenderFunction for torch.autograd.gradcheck (FP64 only here)."""

    @staticmethod
    def forward(ctx, weights64, scene: Scene, o, d, near=None, far=None, max_samples=None):
        weights64 = _dev(weights64, torch.float64, "weights64")
        N = o.shape[1]
        opts = _opts(scene, near, far, max_samples, "fp64")
        ws = torch.empty(int(lib().r360_workspace_bytes(scene._h, N, opts.max_samples)), dtype=torch.uint8,
                         device=o.device)
        rgb = torch.empty(3, N, dtype=torch.float64, device=o.device)
        check(lib().r360_gradcheck_forward(scene._h, _ptr(weights64), _ptr(o), _ptr(d), N, C.byref(opts), _ptr(rgb),
                                           _ptr(ws), ws.numel(), _stream()))
        ctx.scene, ctx.opts, ctx.ws = scene, opts, ws
        ctx.save_for_backward(weights64, o, d)
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        w64, o, d = ctx.saved_tensors
        N = o.shape[1]
        g = torch.empty_like(w64)
        gr = grad_rgb.contiguous().to(torch.float64)
        check(lib().r360_gradcheck_backward(ctx.scene._h, _ptr(w64), _ptr(o), _ptr(d), N, C.byref(ctx.opts),
                                            _ptr(gr), _ptr(g), _ptr(ctx.ws), ctx.ws.numel(), _stream()))
        return g, None, None, None, None, None, None
