"""Seeded synthetic inputs for the 360Roam hot path.

This module is the only code shared by the FP64 oracle side and the HIP side
of the tests and the benchmark. It draws random numbers and lays out input
arrays (occupancy grids, field-assignment maps, packed MLP weights, camera
centres, ray draws, targets). It holds none of the method's arithmetic: no
ray generation (Eq.2/Eq.3), no sampling, no encoding, no MLP and no
compositing. Random numbers the method needs are passed in as arrays.

Generator
---------
Counter-based SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the value for
(seed, stream, index) is the SplitMix64 output function applied to
``key(seed, stream) + (index + 1) * 0x9E3779B97F4A7C15`` (mod 2**64), where
``key`` is the output function applied to ``seed * K1 ^ stream * K2``.
A uniform in [0, 1) is ``(z >> 40) * 2**-24`` (exact in FP32); a normal is
Box-Muller in FP64 on two uniforms with 53 bits each.

Streams: 0 scene, 1 field map, 2 weights, 3 teacher weights, 4 cameras,
5 ray draws, 6 noise. The master seed is 0x360 unless overridden.

Scenes follow the synthetic stand-ins for the paper's indoor dataset
(Sec. 6, 10 real scenes that are not available): a box [-4, 4]^3 m holding
walls and furniture as solid axis-aligned boxes plus salt noise, split into
local fields either round-robin, by an octree with a bounded number of
occupied voxels per leaf, or by Zipf-distributed runs in Morton order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field
from typing import List, Optional

import numpy as np

MASTER_SEED = 0x360
STREAM_SCENE, STREAM_FIELDS, STREAM_WEIGHTS, STREAM_TEACHER, STREAM_CAMERAS, STREAM_RAYS, STREAM_NOISE = range(7)

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_K1 = np.uint64(0xD1B54A32D192ED03)
_K2 = np.uint64(0xABC98388FB8FAC03)


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def u64(seed: int, stream: int, index) -> np.ndarray:
    """Raw 64-bit draws for the given counter indices."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = _mix(np.array([np.uint64(seed) * _K1 ^ np.uint64(stream) * _K2], dtype=np.uint64))[0]
        z = key + (idx + np.uint64(1)) * _GOLDEN
    return _mix(z)


def uniform(seed: int, stream: int, index) -> np.ndarray:
    """U[0,1) with 24 random bits, returned as float64 (exact in float32)."""
    return (u64(seed, stream, index) >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)


def uniform53(seed: int, stream: int, index) -> np.ndarray:
    return (u64(seed, stream, index) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, stream: int, index) -> np.ndarray:
    """Standard normal by Box-Muller on the draw pair (2i, 2i+1)."""
    idx = np.asarray(index, dtype=np.uint64)
    u1 = 1.0 - uniform53(seed, stream, idx * np.uint64(2))
    u2 = uniform53(seed, stream, idx * np.uint64(2) + np.uint64(1))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def randint(seed: int, stream: int, index, lo: int, hi: int) -> np.ndarray:
    """Uniform integers in [lo, hi] (inclusive)."""
    u = uniform53(seed, stream, index)
    return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64)


# ----------------------------------------------------------------------------
# MLP parameter layout (canonical FP32 order, row-major [out x in] matrices)
# ----------------------------------------------------------------------------

def pe_dim(L: int) -> int:
    """Width of the per-component positional encoding with the identity term."""
    return 3 + 6 * L


def local_mlp_layout(hidden: int, L_xyz: int = 10, L_dir: int = 4):
    """(name, shape) list of one local field's tensors in canonical order.

    W1[h x 63], b1, W2[h x h], b2, w_sigma[1 x h], b_sigma, Wf[h x h], bf,
    W3[h x (h + 27)], b3, W4[3 x h], b4; W3's input order is [f ; gamma(d)].
    """
    h, dx, dd = hidden, pe_dim(L_xyz), pe_dim(L_dir)
    return [("W1", (h, dx)), ("b1", (h,)), ("W2", (h, h)), ("b2", (h,)),
            ("ws", (1, h)), ("bs", (1,)), ("Wf", (h, h)), ("bf", (h,)),
            ("W3", (h, h + dd)), ("b3", (h,)), ("W4", (3, h)), ("b4", (3,))]


def global_mlp_layout(width: int = 256, L_xyz: int = 10, L_dir: int = 4, color_width: int = 128):
    """(name, shape) list of the global omnidirectional field's tensors.

    Eight position layers with the encoded position concatenated again at the
    fifth layer input, a density head and a feature layer, then the colour
    branch on [feature ; gamma(d)] (the 360NeRF architecture table).
    """
    w, dx, dd, c = width, pe_dim(L_xyz), pe_dim(L_dir), color_width
    lay = [("W1", (w, dx)), ("b1", (w,))]
    for k in (2, 3, 4):
        lay += [(f"W{k}", (w, w)), (f"b{k}", (w,))]
    lay += [("W5", (w, w + dx)), ("b5", (w,))]
    for k in (6, 7, 8):
        lay += [(f"W{k}", (w, w)), (f"b{k}", (w,))]
    lay += [("ws", (1, w)), ("bs", (1,)), ("Wf", (w, w)), ("bf", (w,)),
            ("W10", (c, w + dd)), ("b10", (c,)), ("W11", (3, c)), ("b11", (3,))]
    return lay


def n_params(layout) -> int:
    return int(sum(int(np.prod(s)) for _, s in layout))


def xavier_weights(layout, n_nets: int, seed: int, stream: int) -> np.ndarray:
    """[n_nets, P] float32: Xavier-uniform matrices, zero biases."""
    P = n_params(layout)
    out = np.zeros((n_nets, P), dtype=np.float32)
    idx = 0
    for name, shape in layout:
        size = int(np.prod(shape))
        if len(shape) == 2:
            fan_out, fan_in = shape
            a = math.sqrt(6.0 / (fan_in + fan_out))
            counter = np.arange(n_nets * P, dtype=np.uint64).reshape(n_nets, P)[:, idx:idx + size]
            u = uniform(seed, stream, counter)
            out[:, idx:idx + size] = ((2.0 * u - 1.0) * a).astype(np.float32)
        idx += size
    return out


def unpack(layout, flat: np.ndarray) -> dict:
    """Views of a flat parameter vector as named arrays."""
    res, idx = {}, 0
    for name, shape in layout:
        size = int(np.prod(shape))
        res[name] = flat[idx:idx + size].reshape(shape)
        idx += size
    return res


# ----------------------------------------------------------------------------
# Scenes
# ----------------------------------------------------------------------------

@dataclass
class Scene:
    n: int                      # voxels per axis (cubic grid)
    lo: float                   # lower corner on every axis (m)
    voxel: float                # voxel edge (m), a power of two
    occ: np.ndarray             # float32 [n, n, n] occupancy probability, x fastest ([z][y][x])
    threshold: float            # occupied where occ > threshold
    field_map: np.ndarray       # int32 [n, n, n], -1 = no field
    n_fields: int
    hidden: int
    weights: np.ndarray         # float32 [n_fields, P] canonical order
    L_xyz: int = 10
    L_dir: int = 4
    center: tuple = (0.0, 0.0, 0.0)
    half_extent: float = 4.0
    near: float = 0.0
    far: float = float("inf")
    max_samples: int = 32
    samples_per_voxel: int = 1  # samples per occupied voxel segment
    frames: Optional[np.ndarray] = None   # per-field encoding frames [n_fields, 4] (centre, half extent)
    name: str = ""
    meta: dict = dc_field(default_factory=dict)

    @property
    def occupied(self) -> np.ndarray:
        return self.occ > np.float32(self.threshold)

    @property
    def n_params(self) -> int:
        return n_params(local_mlp_layout(self.hidden, self.L_xyz, self.L_dir))


def _boxes(seed: int, n: int, scale: int) -> np.ndarray:
    """Solid boxes: 4 vertical walls and 8 furniture pieces (voxel indices)."""
    occ = np.zeros((n, n, n), dtype=bool)  # [z][y][x]
    base = 1 << 40
    k = 0

    def draw(lo, hi):
        nonlocal k
        v = int(randint(seed, STREAM_SCENE, [base + k], lo, hi)[0])
        k += 1
        return v

    for w in range(4):
        thick = draw(2 * scale, 4 * scale)
        e1 = draw(64 * scale, min(128 * scale, n))
        e2 = draw(64 * scale, min(128 * scale, n))
        if w % 2 == 0:     # thin along x, spans y and z
            sx, sy, sz = thick, e1, e2
        else:              # thin along z
            sx, sy, sz = e1, e2, thick
        x0 = draw(0, n - sx); y0 = draw(0, n - sy); z0 = draw(0, n - sz)
        occ[z0:z0 + sz, y0:y0 + sy, x0:x0 + sx] = True
    for f in range(8):
        sx = draw(6 * scale, 24 * scale); sy = draw(6 * scale, 24 * scale); sz = draw(6 * scale, 24 * scale)
        x0 = draw(0, n - sx); y0 = draw(0, n - sy); z0 = draw(0, n - sz)
        occ[z0:z0 + sz, y0:y0 + sy, x0:x0 + sx] = True
    return occ


def _salt(seed: int, n: int, rate: float) -> np.ndarray:
    out = np.empty(n * n * n, dtype=bool)
    step = 1 << 22
    for s in range(0, n * n * n, step):
        e = min(s + step, n * n * n)
        out[s:e] = uniform(seed, STREAM_SCENE, np.arange(s, e, dtype=np.uint64)) < rate
    return out.reshape(n, n, n)


def octree_fields(occ: np.ndarray, max_per_leaf: int) -> np.ndarray:
    """Recursive octree split until a node holds <= max_per_leaf occupied voxels.

    Leaves with at least one occupied voxel become fields, numbered in
    depth-first order over children (x bit 0, y bit 1, z bit 2). Only occupied
    voxels receive a field id.
    """
    n = occ.shape[0]
    cs = np.zeros((n + 1, n + 1, n + 1), dtype=np.int64)
    cs[1:, 1:, 1:] = occ.astype(np.int64).cumsum(0).cumsum(1).cumsum(2)

    def count(x0, y0, z0, s):
        x1, y1, z1 = x0 + s, y0 + s, z0 + s
        return int(cs[z1, y1, x1] - cs[z0, y1, x1] - cs[z1, y0, x1] - cs[z1, y1, x0]
                   + cs[z0, y0, x1] + cs[z0, y1, x0] + cs[z1, y0, x0] - cs[z0, y0, x0])

    fmap = np.full(occ.shape, -1, dtype=np.int32)
    nf = 0
    stack = [(0, 0, 0, n)]
    while stack:
        x0, y0, z0, s = stack.pop()
        c = count(x0, y0, z0, s)
        if c == 0:
            continue
        if c <= max_per_leaf or s == 1:
            sub = occ[z0:z0 + s, y0:y0 + s, x0:x0 + s]
            blk = fmap[z0:z0 + s, y0:y0 + s, x0:x0 + s]
            blk[sub] = nf
            nf += 1
            continue
        h = s // 2
        for child in reversed(range(8)):   # pushed reversed so child 0 is visited first
            stack.append((x0 + h * (child & 1), y0 + h * ((child >> 1) & 1), z0 + h * ((child >> 2) & 1), h))
    return fmap


def morton3(x: np.ndarray, y: np.ndarray, z: np.ndarray) -> np.ndarray:
    def spread(v):
        v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
        v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
        v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
        return v
    return spread(x) | (spread(y) << np.uint64(1)) | (spread(z) << np.uint64(2))


def zipf_fields(occ: np.ndarray, n_fields: int, exponent: float) -> np.ndarray:
    """Contiguous runs of occupied voxels in Morton order, sizes ~ k^-exponent."""
    zz, yy, xx = np.nonzero(occ)
    order = np.argsort(morton3(xx, yy, zz), kind="stable")
    S = len(order)
    share = np.arange(1, n_fields + 1, dtype=np.float64) ** (-exponent)
    share /= share.sum()
    sizes = np.maximum(1, np.floor(share * S).astype(np.int64))
    sizes[0] += S - sizes.sum()
    assert sizes.min() >= 1 and sizes.sum() == S
    labels = np.repeat(np.arange(n_fields, dtype=np.int32), sizes)
    fmap = np.full(occ.shape, -1, dtype=np.int32)
    fmap[zz[order], yy[order], xx[order]] = labels
    return fmap


def scene_small(seed: int = MASTER_SEED) -> Scene:
    """256x128 correctness scene: 32^3 grid, p ~ U(0,1), occupied where
    p > 0.7, occupied voxels assigned round-robin (k-th in linear order -> k mod 8)
    to 8 fields of hidden width 32; up to 32 samples per ray."""
    n = 32
    occ = uniform(seed, STREAM_SCENE, np.arange(n ** 3, dtype=np.uint64)).astype(np.float32).reshape(n, n, n)
    thr = 0.7
    fmap = np.full((n, n, n), -1, dtype=np.int32)
    occupied = (occ > np.float32(thr)).reshape(-1)
    f = fmap.reshape(-1)
    f[occupied] = (np.arange(int(occupied.sum())) % 8).astype(np.int32)
    lay = local_mlp_layout(32)
    w = xavier_weights(lay, 8, seed, STREAM_WEIGHTS)
    return Scene(n=n, lo=-4.0, voxel=0.25, occ=occ, threshold=thr, field_map=fmap, n_fields=8,
                 hidden=32, weights=w, near=0.0, far=float("inf"), max_samples=32, name="equirect-256x128")


def _room_occupancy(seed: int, n: int, scale: int, salt: float) -> np.ndarray:
    return _boxes(seed, n, scale) | _salt(seed, n, salt)


def scene_room(seed: int = MASTER_SEED, with_weights: bool = True) -> Scene:
    """2048x1024 headline scene: 128^3 grid of 12 solid boxes (4 walls,
    8 furniture) plus 2% salt noise; octree split to <= 4096 occupied voxels
    per leaf; hidden width 64; up to 64 samples per ray, near 0.05 m, far 12 m."""
    n = 128
    occb = _room_occupancy(seed, n, 1, 0.02)
    fmap = octree_fields(occb, 4096)
    nf = int(fmap.max()) + 1
    occ = occb.astype(np.float32)
    lay = local_mlp_layout(64)
    w = xavier_weights(lay, nf, seed, STREAM_WEIGHTS) if with_weights else np.zeros((nf, n_params(lay)), np.float32)
    return Scene(n=n, lo=-4.0, voxel=0.0625, occ=occ, threshold=0.5, field_map=fmap, n_fields=nf,
                 hidden=64, weights=w, near=0.05, far=12.0, max_samples=64, name="equirect-2048x1024")


def scene_large(seed: int = MASTER_SEED) -> Scene:
    """Large uneven scene: 256^3 grid (the room generator scaled x2), 512
    fields with Zipf(1.2) occupied-voxel counts, hidden 64, up to 96 samples."""
    n = 256
    occb = _room_occupancy(seed, n, 2, 0.02)
    fmap = zipf_fields(occb, 512, 1.2)
    lay = local_mlp_layout(64)
    w = xavier_weights(lay, 512, seed, STREAM_WEIGHTS)
    return Scene(n=n, lo=-4.0, voxel=0.03125, occ=occb.astype(np.float32), threshold=0.5, field_map=fmap,
                 n_fields=512, hidden=64, weights=w, near=0.05, far=12.0, max_samples=96,
                 name="large-uneven-256")


def teacher_weights(scene: Scene, seed: int = MASTER_SEED) -> np.ndarray:
    return xavier_weights(local_mlp_layout(scene.hidden, scene.L_xyz, scene.L_dir), scene.n_fields,
                          seed, STREAM_TEACHER)


def tiny_scene(n: int, seed: int, p_occ: float = 0.5, n_fields: int = 3, hidden: int = 32,
               max_samples: int = 32, near: float = 0.0, far: float = float("inf")) -> Scene:
    """Small random grid over [-4,4]^3 for brute-force checks."""
    occ = uniform(seed, STREAM_SCENE, np.arange(n ** 3, dtype=np.uint64)).astype(np.float32).reshape(n, n, n)
    thr = np.float32(1.0 - p_occ)
    fmap = np.full((n, n, n), -1, dtype=np.int32)
    occupied = (occ > thr).reshape(-1)
    fmap.reshape(-1)[occupied] = (np.arange(int(occupied.sum())) % n_fields).astype(np.int32)
    lay = local_mlp_layout(hidden)
    w = xavier_weights(lay, n_fields, seed, STREAM_WEIGHTS)
    vox = 8.0 / n
    return Scene(n=n, lo=-4.0, voxel=vox, occ=occ, threshold=float(thr), field_map=fmap, n_fields=n_fields,
                 hidden=hidden, weights=w, near=near, far=far, max_samples=max_samples, name=f"tiny-{n}")


# ----------------------------------------------------------------------------
# Cameras and ray draws
# ----------------------------------------------------------------------------

IDENTITY_C2W = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], dtype=np.float32)


def c2w_at(center) -> np.ndarray:
    """Row-major 3x4 camera-to-world with R = I and the given centre."""
    m = IDENTITY_C2W.copy()
    m[3], m[7], m[11] = center
    return m


def c2w_yaw(center, quarter_turns: int) -> np.ndarray:
    """Rotation about the y axis by quarter_turns * 90 degrees (entries 0/+-1)."""
    c, s = [(1, 0), (0, 1), (-1, 0), (0, -1)][quarter_turns % 4]
    m = np.array([c, 0, s, center[0], 0, 1, 0, center[1], -s, 0, c, center[2]], dtype=np.float32)
    return m


def camera_centres(scene: Scene, count: int, seed: int = MASTER_SEED, lim: float = 3.5) -> np.ndarray:
    """Camera centres uniform in [-lim, lim]^3, rejecting occupied voxels."""
    out = []
    k = 0
    occ = scene.occupied
    while len(out) < count:
        p = (2.0 * uniform(seed, STREAM_CAMERAS, np.arange(3 * k, 3 * k + 3, dtype=np.uint64)) - 1.0) * lim
        p = p.astype(np.float32)
        k += 1
        ix = np.floor((p.astype(np.float64) - scene.lo) / scene.voxel).astype(np.int64)
        if np.all((ix >= 0) & (ix < scene.n)) and occ[ix[2], ix[1], ix[0]]:
            continue
        out.append(p)
    return np.stack(out).astype(np.float32)


def ray_draws(n_rays: int, n_cams: int, W: int, H: int, seed: int = MASTER_SEED):
    """(camera index, pixel u, pixel v) per ray, each uniform."""
    i = np.arange(n_rays, dtype=np.uint64)
    cam = randint(seed, STREAM_RAYS, i * np.uint64(3), 0, n_cams - 1).astype(np.int32)
    u = randint(seed, STREAM_RAYS, i * np.uint64(3) + np.uint64(1), 0, W - 1).astype(np.int32)
    v = randint(seed, STREAM_RAYS, i * np.uint64(3) + np.uint64(2), 0, H - 1).astype(np.int32)
    return cam, u, v


def noise(n: int, std: float, seed: int = MASTER_SEED) -> np.ndarray:
    return (std * normal(seed, STREAM_NOISE, np.arange(n, dtype=np.uint64)))


def random_unit_dirs(n: int, seed: int, stream: int = STREAM_RAYS) -> np.ndarray:
    """[3, n] float32 directions from normalised Gaussian triples (input draws only)."""
    g = normal(seed, stream, np.arange(3 * n, dtype=np.uint64)).reshape(n, 3)
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return np.ascontiguousarray(g.T.astype(np.float32))


def occupancy_measurements(n: int, seed: int, d_lo: float = 0.2, d_hi: float = 8.0, u_max: float = 0.5,
                           p_valid: float = 0.8):
    """Synthetic per-ray (depth, uncertainty, opacity) for the Stage I update
    (input draws only): depth U[d_lo, d_hi), uncertainty U[0, u_max), and an
    opacity of 1 for a fraction p_valid of the rays, else U[0, 1/2)."""
    idx = np.arange(4 * n, dtype=np.uint64)
    u = uniform(seed, STREAM_NOISE, idx).reshape(4, n)
    depth = (d_lo + (d_hi - d_lo) * u[0]).astype(np.float32)
    uncert = (u_max * u[1]).astype(np.float32)
    opacity = np.where(u[2] < p_valid, 1.0, 0.5 * u[3]).astype(np.float32)
    return depth, uncert, opacity


def field_points(scene: Scene, per_field: int, seed: int):
    """Distillation points (input draws only): per field, per_field voxels of
    that field chosen uniformly with replacement, a uniform position inside
    each, and a uniform unit view direction. Returns x [3, M], d [3, M],
    field [M] (int32), grouped by field."""
    fm = scene.field_map.reshape(-1)
    order = np.argsort(fm, kind="stable")
    counts = np.bincount(fm[fm >= 0], minlength=scene.n_fields)
    starts = np.concatenate([[0], np.cumsum(counts)]) + int((fm < 0).sum())
    M = per_field * scene.n_fields
    u = uniform(seed, STREAM_RAYS, np.arange(4 * M, dtype=np.uint64)).reshape(4, M)
    field = np.repeat(np.arange(scene.n_fields, dtype=np.int32), per_field)
    pick = starts[field] + np.minimum((u[0] * counts[field]).astype(np.int64), counts[field] - 1)
    lin = order[pick]
    n = scene.n
    ijk = np.stack([lin % n, (lin // n) % n, lin // (n * n)]).astype(np.float64)
    x = (scene.lo + (ijk + u[1:4]) * scene.voxel).astype(np.float32)
    d = random_unit_dirs(M, seed + 1)
    return np.ascontiguousarray(x), d, field
