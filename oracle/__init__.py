"""FP64 CPU oracle for the 360Roam hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path (the HIP library and
its Python binding) never imports, links or calls it.

This module is a thin ctypes wrapper over ``oracle.cpp`` (plain C++17 loops,
FP64 after a specified FP32 geometric front end). The equations each
function follows are cited in ``oracle.cpp``.

Parity pins (what fixes the oracle independently of itself) live in
``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread"]


def build(force: bool = True, out: Optional[str] = None, plant: int = 0) -> str:
    """Compile oracle.cpp with g++ (no contraction, no fast-math). `plant`
    (tests only) builds a copy with a deliberate mistake into `out`."""
    target = out or _LIB
    if force or not os.path.exists(target):
        tmp = target + ".tmp"
        extra = [f"-DORC_PLANT={plant}"] if plant else []
        subprocess.check_call(["g++", *CXXFLAGS, *extra, _SRC, "-o", tmp])
        os.replace(tmp, target)
    return target


def use_library(path: Optional[str]):
    """Point this module at another build of the oracle (tests only); None
    restores the default build."""
    global _lib, _LIB_OVERRIDE
    _LIB_OVERRIDE = path
    _lib = None


_LIB_OVERRIDE: Optional[str] = None


class OrcScene(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("lo", C.c_float * 3), ("voxel", C.c_float), ("threshold", C.c_float),
                ("occ", C.c_void_p), ("field", C.c_void_p), ("n_fields", C.c_int32), ("hidden", C.c_int32),
                ("L_xyz", C.c_int32), ("L_dir", C.c_int32), ("center", C.c_float * 3), ("half_extent", C.c_float),
                ("weights", C.c_void_p), ("near_", C.c_float), ("far_", C.c_float), ("max_samples", C.c_int32),
                ("samples_per_voxel", C.c_int32), ("frames", C.c_void_p)]


class OrcGlobal(C.Structure):
    _fields_ = [("width", C.c_int32), ("color_width", C.c_int32), ("L_xyz", C.c_int32), ("L_dir", C.c_int32),
                ("n_samples", C.c_int32), ("near_", C.c_float), ("far_", C.c_float), ("center", C.c_float * 3),
                ("half_extent", C.c_float), ("weights", C.c_void_p), ("n", C.c_int32 * 3), ("lo", C.c_float * 3),
                ("voxel", C.c_float)]


class OrcOcc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("lo", C.c_float * 3), ("voxel", C.c_float), ("near_", C.c_float),
                ("far_", C.c_float), ("l_hit", C.c_float), ("l_miss", C.c_float), ("l_min", C.c_float),
                ("l_max", C.c_float), ("min_opacity", C.c_float)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _LIB_OVERRIDE or _LIB
        if not os.path.exists(path):
            build()
        L = C.CDLL(path)
        vp, i32, i64, f32, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
        sig = {
            "orc_equirect_lut": (None, [C.c_int, C.c_int, vp, vp, vp, vp]),
            "orc_equirect_rays": (None, [C.c_int, C.c_int, vp, vp, i64, vp, vp]),
            "orc_pinhole_rays": (None, [C.c_int, C.c_int, f32, f32, vp, i64, i64, vp, vp]),
            "orc_ods_rays": (None, [C.c_int, C.c_int, vp, f32, vp, i64, vp, vp]),
            "orc_field_frames": (None, [vp, vp, f32, vp, i32, vp]),
            "orc_count_samples": (None, [vp, i64, vp, vp, vp, C.c_int]),
            "orc_sample_rays": (None, [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int]),
            "orc_encode": (None, [vp, C.c_int, vp]),
            "orc_local_mlp": (None, [vp, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp]),
            "orc_composite": (None, [C.c_int, vp, vp, vp, vp, vp, vp, vp, vp]),
            "orc_composite_backward": (None, [C.c_int, vp, vp, vp, vp, vp, vp]),
            "orc_render_rays": (None, [vp, i64, vp, vp, vp, vp, vp, C.c_int]),
            "orc_sample_outputs": (None, [vp, i64, vp, vp, vp, vp, vp, i64, C.c_int]),
            "orc_train_grad": (f64, [vp, i64, vp, vp, vp, vp, vp, C.c_int, vp, f64, vp]),
            "orc_invdepth_t": (None, [C.c_int, f32, f32, vp, vp]),
            "orc_global_step": (f64, [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int]),
            "orc_global_mlp": (None, [vp, C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp]),
            "orc_local_params": (i64, [C.c_int, C.c_int, C.c_int]),
            "orc_global_params": (i64, [C.c_int, C.c_int, C.c_int, C.c_int]),
            "orc_adam": (None, [i64, vp, vp, vp, vp, i64, f64, f64, f64, f64]),
            "orc_depth_stats": (None, [i64, C.c_int, vp, vp, vp, vp, vp, vp]),
            "orc_occupancy_update": (None, [vp, vp, vp, i64, vp, vp, vp, vp, vp, C.c_int]),
            "orc_global_measure": (None, [vp, i64, vp, vp, vp, vp, vp, C.c_int]),
            "orc_assign_fields": (i64, [vp, vp, f32, i32, vp]),
            "orc_distill": (f64, [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int]),
            "orc_global_points": (None, [vp, i64, vp, vp, vp, vp, C.c_int]),
            "orc_assign_uniform": (i32, [vp, vp, f32, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


class SceneHandle:
    """Keeps the arrays referenced by an OrcScene alive."""

    def __init__(self, scene, weights: Optional[np.ndarray] = None, max_samples: Optional[int] = None,
                 near: Optional[float] = None, far: Optional[float] = None):
        self.occ = _c(scene.occ, np.float32)
        self.field = _c(scene.field_map, np.int32)
        self.weights = _c(scene.weights if weights is None else weights, np.float32)
        s = OrcScene()
        s.n[:] = [scene.n] * 3
        s.lo[:] = [scene.lo] * 3
        s.voxel = scene.voxel
        s.threshold = scene.threshold
        s.occ = self.occ.ctypes.data
        s.field = self.field.ctypes.data
        s.n_fields = scene.n_fields
        s.hidden = scene.hidden
        s.L_xyz, s.L_dir = scene.L_xyz, scene.L_dir
        s.center[:] = list(scene.center)
        s.half_extent = scene.half_extent
        s.weights = self.weights.ctypes.data
        s.near_ = scene.near if near is None else near
        s.far_ = scene.far if far is None else far
        s.max_samples = scene.max_samples if max_samples is None else max_samples
        s.samples_per_voxel = getattr(scene, "samples_per_voxel", 1)
        fr = getattr(scene, "frames", None)
        self.frames = None if fr is None else _c(fr, np.float32)
        s.frames = None if self.frames is None else self.frames.ctypes.data
        self.s = s

    @property
    def ptr(self):
        return C.byref(self.s)


# ---------------------------------------------------------------------------
# Rays
# ---------------------------------------------------------------------------

def equirect_lut(W: int, H: int):
    sphi = np.empty(W, np.float32); cphi = np.empty(W, np.float32)
    sth = np.empty(H, np.float32); cth = np.empty(H, np.float32)
    lib().orc_equirect_lut(W, H, _p(sphi), _p(cphi), _p(sth), _p(cth))
    return sphi, cphi, sth, cth


def equirect_rays(W: int, H: int, c2w: np.ndarray, pix: Optional[np.ndarray] = None):
    """o, d as [3, N] float32 for pixels (linear v*W+u) or the whole image."""
    c2w = _c(c2w, np.float32)
    if pix is None:
        N = W * H
        pp = None
    else:
        pix = _c(pix, np.int64)
        N = len(pix)
        pp = _p(pix)
    o = np.empty((3, N), np.float32); d = np.empty((3, N), np.float32)
    lib().orc_equirect_rays(W, H, _p(c2w), pp, N, _p(o), _p(d))
    return o, d


def ods_rays(W: int, H: int, c2w: np.ndarray, eye: float, pix: Optional[np.ndarray] = None):
    """Omni-directional stereo rays of one eye (eye = signed half inter-pupillary distance)."""
    c2w = _c(c2w, np.float32)
    N = W * H if pix is None else len(pix)
    pix_a = None if pix is None else _c(pix, np.int64)
    o = np.empty((3, N), np.float32); d = np.empty((3, N), np.float32)
    lib().orc_ods_rays(W, H, _p(c2w), eye, None if pix_a is None else _p(pix_a), N, _p(o), _p(d))
    return o, d


def pinhole_rays(W: int, H: int, fx: float, fy: float, c2w: np.ndarray, start: int = 0, count: Optional[int] = None):
    c2w = _c(c2w, np.float32)
    N = W * H - start if count is None else count
    o = np.empty((3, N), np.float32); d = np.empty((3, N), np.float32)
    lib().orc_pinhole_rays(W, H, fx, fy, _p(c2w), start, N, _p(o), _p(d))
    return o, d


# ---------------------------------------------------------------------------
# Sampling
# ---------------------------------------------------------------------------

def sample_rays(scene, o: np.ndarray, d: np.ndarray, threads: Optional[int] = None, **kw):
    """Ray-major sample lists: dict(counts, offsets[N+1], t_mid, delta, ray_id, voxel, field)."""
    h = SceneHandle(scene, **kw)
    o = _c(o, np.float32); d = _c(d, np.float32)
    N = o.shape[1]
    nt = threads or default_threads()
    counts = np.empty(N, np.int32)
    lib().orc_count_samples(h.ptr, N, _p(o), _p(d), _p(counts), nt)
    offsets = np.zeros(N + 1, np.int64)
    np.cumsum(counts, out=offsets[1:])
    S = int(offsets[-1])
    t_mid = np.empty(S, np.float32); delta = np.empty(S, np.float32)
    ray_id = np.empty(S, np.int32); voxel = np.empty(S, np.int32); field = np.empty(S, np.int32)
    lib().orc_sample_rays(h.ptr, N, _p(o), _p(d), _p(offsets), _p(t_mid), _p(delta), _p(ray_id), _p(voxel),
                          _p(field), nt)
    return dict(counts=counts, offsets=offsets, t_mid=t_mid, delta=delta, ray_id=ray_id, voxel=voxel, field=field)


# ---------------------------------------------------------------------------
# Encoding / MLP / compositing building blocks
# ---------------------------------------------------------------------------

def encode(x, L: int) -> np.ndarray:
    x = _c(x, np.float64)
    out = np.empty(3 + 6 * L, np.float64)
    lib().orc_encode(_p(x), L, _p(out))
    return out


def local_mlp(weights: np.ndarray, hidden: int, xh, direction, L_xyz: int = 10, L_dir: int = 4):
    w = _c(weights, np.float32)
    xh = _c(xh, np.float64); dr = _c(direction, np.float64)
    sigma = np.zeros(1, np.float64); rgb = np.zeros(3, np.float64)
    lib().orc_local_mlp(_p(w), hidden, L_xyz, L_dir, _p(xh), _p(dr), _p(sigma), _p(rgb))
    return float(sigma[0]), rgb


def global_mlp(weights: np.ndarray, xh, direction, width: int = 256, color_width: int = 128,
               L_xyz: int = 10, L_dir: int = 4):
    w = _c(weights, np.float32)
    xh = _c(xh, np.float64); dr = _c(direction, np.float64)
    sigma = np.zeros(1, np.float64); rgb = np.zeros(3, np.float64)
    lib().orc_global_mlp(_p(w), width, color_width, L_xyz, L_dir, _p(xh), _p(dr), _p(sigma), _p(rgb))
    return float(sigma[0]), rgb


def composite(sigma, rgb, t_mid, delta):
    """Returns (C[3], D, A, w[n]) in FP64."""
    sigma = _c(sigma, np.float64); rgb = _c(rgb, np.float64).reshape(-1, 3)
    t_mid = _c(t_mid, np.float64); delta = _c(delta, np.float64)
    n = len(sigma)
    Cc = np.zeros(3); D = np.zeros(1); A = np.zeros(1); w = np.zeros(max(n, 1))
    lib().orc_composite(n, _p(sigma), _p(rgb), _p(t_mid), _p(delta), _p(Cc), _p(D), _p(A), _p(w))
    return Cc, float(D[0]), float(A[0]), w[:n]


def composite_backward(sigma, rgb, delta, g):
    sigma = _c(sigma, np.float64); rgb = _c(rgb, np.float64).reshape(-1, 3)
    delta = _c(delta, np.float64); g = _c(g, np.float64)
    n = len(sigma)
    ds = np.zeros(max(n, 1)); dc = np.zeros((max(n, 1), 3))
    lib().orc_composite_backward(n, _p(sigma), _p(rgb), _p(delta), _p(g), _p(ds), _p(dc))
    return ds[:n], dc[:n]


def local_params(hidden: int, L_xyz: int = 10, L_dir: int = 4) -> int:
    return int(lib().orc_local_params(hidden, L_xyz, L_dir))


def global_params(width: int = 256, color_width: int = 128, L_xyz: int = 10, L_dir: int = 4) -> int:
    return int(lib().orc_global_params(width, color_width, L_xyz, L_dir))


# ---------------------------------------------------------------------------
# Full paths
# ---------------------------------------------------------------------------

def render_rays(scene, o, d, threads: Optional[int] = None, **kw):
    """(rgb [3, N], depth [N], opacity [N]) in FP64."""
    h = SceneHandle(scene, **kw)
    o = _c(o, np.float32); d = _c(d, np.float32)
    N = o.shape[1]
    rgb = np.empty((3, N)); depth = np.empty(N); opac = np.empty(N)
    lib().orc_render_rays(h.ptr, N, _p(o), _p(d), _p(rgb), _p(depth), _p(opac), threads or default_threads())
    return rgb, depth, opac


def render_rays_terminated(scene, o, d, term_eps: float, term_after: int, threads: Optional[int] = None, **kw):
    """Early ray termination as a stopping rule of volume rendering: a ray
    stops after its first term_after samples when its transmittance there,
    exp(-sum tau) = 1 - (opacity of those samples), is below term_eps, and
    keeps all its samples otherwise. Returns (rgb, depth, opacity, stopped)
    in FP64; stopped marks the rays that stopped with samples left."""
    full = render_rays(scene, o, d, threads, **kw)
    first = render_rays(scene, o, d, threads, **dict(kw, max_samples=term_after))
    counts = np.diff(sample_rays(scene, o, d, **kw)["offsets"])
    T = 1.0 - first[2]
    stopped = (counts > term_after) & (T < term_eps)
    rgb = np.where(stopped[None, :], first[0], full[0])
    depth = np.where(stopped, first[1], full[1])
    opac = np.where(stopped, first[2], full[2])
    return rgb, depth, opac, stopped


def sample_outputs(scene, o, d, offsets, threads: Optional[int] = None, **kw):
    """Per-sample sigma [S] and rgb [3, S] in ray-major order."""
    h = SceneHandle(scene, **kw)
    o = _c(o, np.float32); d = _c(d, np.float32)
    offsets = _c(offsets, np.int64)
    N = o.shape[1]
    S = int(offsets[-1])
    sigma = np.empty(S); rgb = np.empty((3, S))
    lib().orc_sample_outputs(h.ptr, N, _p(o), _p(d), _p(offsets), _p(sigma), _p(rgb), S, threads or default_threads())
    return sigma, rgb


def train_grad(scene, o, d, target, weights: Optional[np.ndarray] = None, threads: Optional[int] = None,
               magnitude: bool = False, kink: Optional[float] = None, **kw):
    """(loss, grad [n_fields, P] FP64, rgb [3, N]) for L = mean over rays and
    channels of (C - C*)^2. With magnitude=True a fourth item: the magnitude
    of every gradient entry (the same computation with the absolute value of
    each operand; |grad| <= magnitude), the scale a rounding error of another
    implementation is measured against. With kink = tau as well, a fifth: the
    magnitude of the terms that pass through a ReLU unit whose pre-activation
    lies within tau of zero (a computation with pre-activation errors up to
    tau may take the other branch there and add or drop such a term whole)."""
    h = SceneHandle(scene, weights=weights, **kw)
    o = _c(o, np.float32); d = _c(d, np.float32); target = _c(target, np.float32)
    N = o.shape[1]
    grad = np.empty(h.weights.shape, np.float64)
    mag = np.empty(h.weights.shape, np.float64) if magnitude else None
    kin = np.empty(h.weights.shape, np.float64) if magnitude and kink is not None else None
    rgb = np.empty((3, N))
    loss = lib().orc_train_grad(h.ptr, N, _p(o), _p(d), _p(target), _p(grad), _p(rgb), threads or default_threads(),
                                _p(mag) if magnitude else None, float(kink or 0.0),
                                _p(kin) if kin is not None else None)
    if kin is not None:
        return float(loss), grad, rgb, mag, kin
    if magnitude:
        return float(loss), grad, rgb, mag
    return float(loss), grad, rgb


def invdepth_t(n_samples: int, near: float, far: float):
    t = np.empty(n_samples, np.float32); delta = np.empty(n_samples, np.float32)
    lib().orc_invdepth_t(n_samples, near, far, _p(t), _p(delta))
    return t, delta


def _global_desc(w, n_samples, near, far, width, color_width, L_xyz, L_dir, center, half_extent, grid_n, grid_lo,
                 voxel):
    g = OrcGlobal()
    g.width, g.color_width, g.L_xyz, g.L_dir, g.n_samples = width, color_width, L_xyz, L_dir, n_samples
    g.near_, g.far_ = near, far
    g.center[:] = list(center)
    g.half_extent = half_extent
    g.weights = w.ctypes.data
    g.n[:] = [grid_n] * 3
    g.lo[:] = [grid_lo] * 3
    g.voxel = voxel
    return g


def global_step(weights, o, d, target, n_samples=128, near=0.1, far=20.0, width=256, color_width=128,
                L_xyz=10, L_dir=4, center=(0.0, 0.0, 0.0), half_extent=4.0, grid_n=128, grid_lo=-4.0,
                voxel=0.0625, occupancy=True, threads: Optional[int] = None):
    """Global field forward + backward; returns dict(loss, grad, rgb, depth, opacity, occ_max)."""
    w = _c(weights, np.float32)
    o = _c(o, np.float32); d = _c(d, np.float32); target = _c(target, np.float32)
    N = o.shape[1]
    g = _global_desc(w, n_samples, near, far, width, color_width, L_xyz, L_dir, center, half_extent, grid_n, grid_lo,
                     voxel)
    grad = np.empty(len(w), np.float64)
    rgb = np.empty((3, N)); depth = np.empty(N); opac = np.empty(N)
    occ = np.zeros(grid_n ** 3, np.float64) if occupancy else None
    loss = lib().orc_global_step(C.byref(g), N, _p(o), _p(d), _p(target), _p(grad), _p(rgb), _p(depth), _p(opac),
                                 _p(occ) if occ is not None else None, threads or default_threads())
    return dict(loss=float(loss), grad=grad, rgb=rgb, depth=depth, opacity=opac,
                occ_max=None if occ is None else occ.reshape(grid_n, grid_n, grid_n))


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.99, eps=1e-8):
    """In-place FP64 Adam update on float64 arrays."""
    for a in (w, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam(len(w), _p(w), _p(g), _p(m), _p(v), step, lr, b1, b2, eps)


# ---- Stage I occupancy (Sec. 4.1, Alg.1) ------------------------------------
def logit(p: float) -> float:
    return float(np.log(p / (1.0 - p)))


def depth_stats(t, delta, sigma):
    """Per-ray (depth, uncertainty, opacity) FP64 from dense [N, S] samples."""
    t = _c(t, np.float32); delta = _c(delta, np.float32); sigma = _c(sigma, np.float32)
    N, S = t.shape
    D = np.empty(N); U = np.empty(N); A = np.empty(N)
    lib().orc_depth_stats(N, S, _p(t), _p(delta), _p(sigma), _p(D), _p(U), _p(A))
    return D, U, A


def occ_desc(n, lo, voxel, near=0.0, far=float("inf"), p_hit=0.7, p_miss=0.4, l_min=-2.0, l_max=3.5,
             min_opacity=0.5) -> OrcOcc:
    g = OrcOcc()
    g.n[:] = list(n) if np.ndim(n) else [n] * 3
    g.lo[:] = list(lo) if np.ndim(lo) else [lo] * 3
    g.voxel = voxel
    g.near_, g.far_ = near, far
    g.l_hit, g.l_miss = logit(p_hit), logit(p_miss)
    g.l_min, g.l_max, g.min_opacity = l_min, l_max, min_opacity
    return g


def occupancy_update(desc: OrcOcc, logit_grid: np.ndarray, o, d, depth, uncert, opacity,
                     threads: Optional[int] = None) -> np.ndarray:
    """One pose's update of the FP32 logit grid [n2, n1, n0] in place; returns the probability grid."""
    assert logit_grid.dtype == np.float32 and logit_grid.flags.c_contiguous
    o = _c(o, np.float32); d = _c(d, np.float32)
    depth = _c(depth, np.float32); uncert = _c(uncert, np.float32); opacity = _c(opacity, np.float32)
    N = o.shape[1]
    prob = np.empty_like(logit_grid)
    lib().orc_occupancy_update(C.byref(desc), _p(logit_grid), _p(prob), N, _p(o), _p(d), _p(depth), _p(uncert),
                               _p(opacity), threads or default_threads())
    return prob


def global_measure(weights, o, d, n_samples=128, near=0.1, far=20.0, width=256, color_width=128, L_xyz=10, L_dir=4,
                   center=(0.0, 0.0, 0.0), half_extent=4.0, threads: Optional[int] = None):
    """Stage I measurement of the global field: per-ray (depth, uncertainty, opacity), FP64."""
    w = _c(weights, np.float32)
    o = _c(o, np.float32); d = _c(d, np.float32)
    N = o.shape[1]
    g = _global_desc(w, n_samples, near, far, width, color_width, L_xyz, L_dir, center, half_extent, 1, 0.0, 1.0)
    D = np.empty(N); U = np.empty(N); A = np.empty(N)
    lib().orc_global_measure(C.byref(g), N, _p(o), _p(d), _p(D), _p(U), _p(A), threads or default_threads())
    return D, U, A


# ---- Stage II field assignment (Sec. 4.2, Alg.1) ----------------------------
def assign_fields(occ: np.ndarray, threshold: float, n_fields: int):
    """(field_map int32 [n2, n1, n0], S) by Alg.1 Stage II."""
    occ = _c(occ, np.float32)
    n = (C.c_int32 * 3)(occ.shape[2], occ.shape[1], occ.shape[0])
    fmap = np.empty(occ.shape, np.int32)
    S = lib().orc_assign_fields(n, _p(occ), threshold, n_fields, _p(fmap))
    return fmap, int(S)


def assign_uniform(occ: np.ndarray, threshold: float, blocks):
    """(field_map, n_fields) for the uniform decomposition into blocks (b0, b1, b2)."""
    occ = _c(occ, np.float32)
    n = (C.c_int32 * 3)(occ.shape[2], occ.shape[1], occ.shape[0])
    b = (C.c_int32 * 3)(*blocks)
    fmap = np.empty(occ.shape, np.int32)
    nf = lib().orc_assign_uniform(n, _p(occ), threshold, b, _p(fmap))
    return fmap, int(nf)


# ---- distillation (Sec. 4.2, Eq.7) -----------------------------------------
def distill(scene, x, d, field, target_sigma, target_rgb, weights: Optional[np.ndarray] = None,
            threads: Optional[int] = None):
    """(loss, grad [n_fields, P] FP64, sigma [M], rgb [3, M]) of the Eq.7 loss summed over fields."""
    h = SceneHandle(scene, weights=weights)
    x = _c(x, np.float32); d = _c(d, np.float32); field = _c(field, np.int32)
    ts = _c(target_sigma, np.float32); tr = _c(target_rgb, np.float32)
    M = x.shape[1]
    grad = np.empty(h.weights.shape, np.float64)
    sig = np.empty(M); rgb = np.empty((3, M))
    loss = lib().orc_distill(h.ptr, M, _p(x), _p(d), _p(field), _p(ts), _p(tr), _p(grad), _p(sig), _p(rgb),
                             threads or default_threads())
    return float(loss), grad, sig, rgb


def global_points(weights, x, d, width=256, color_width=128, L_xyz=10, L_dir=4, center=(0.0, 0.0, 0.0),
                  half_extent=4.0, threads: Optional[int] = None):
    """The global field's (sigma [M], rgb [3, M]) FP64 at points x with directions d ([3, M] each)."""
    w = _c(weights, np.float32)
    x = _c(x, np.float32); d = _c(d, np.float32)
    M = x.shape[1]
    g = _global_desc(w, 2, 0.1, 20.0, width, color_width, L_xyz, L_dir, center, half_extent, 1, 0.0, 1.0)
    sig = np.empty(M); rgb = np.empty((3, M))
    lib().orc_global_points(C.byref(g), M, _p(x), _p(d), _p(sig), _p(rgb), threads or default_threads())
    return sig, rgb


# ---- per-field encoding frames -----------------------------------------------
def field_frames(field_map: np.ndarray, lo, voxel: float, n_fields: int) -> np.ndarray:
    """[n_fields, 4] FP32: the box centre (3) and half extent of each field's voxels."""
    fm = _c(field_map, np.int32)
    n = (C.c_int32 * 3)(fm.shape[2], fm.shape[1], fm.shape[0])
    lo3 = (C.c_float * 3)(*([lo] * 3 if np.ndim(lo) == 0 else list(lo)))
    out = np.empty((n_fields, 4), np.float32)
    lib().orc_field_frames(n, lo3, voxel, _p(fm), n_fields, _p(out))
    return out
