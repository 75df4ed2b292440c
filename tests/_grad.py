"""Helpers for the gradient tests: per-field, per-tensor error measures and
the training-batch ray recipe (20 camera centres in the room scene, pixel
draws uniform over the 2048x1024 view)."""
import numpy as np

import synth


def block_errors(g, ref, layout, floor_frac):
    """Errors of a gradient against its reference, one block per (field,
    tensor). A block's error is max|g - ref| over the block divided by its own
    scale max|ref|; a block whose scale is below floor_frac times the largest
    entry of the whole gradient is measured against that floor instead (its
    entries are rounding-level and carry no relative meaning).

    g, ref: [n_fields, P] (or [P] for one network). Returns a list of
    (error, field, tensor name, block scale), worst first."""
    g = np.atleast_2d(np.asarray(g, np.float64))
    ref = np.atleast_2d(np.asarray(ref, np.float64))
    top = float(np.abs(ref).max())
    floor = floor_frac * top
    out = []
    off = 0
    for name, shape in layout:
        size = int(np.prod(shape))
        d = np.abs(g[:, off:off + size] - ref[:, off:off + size]).max(axis=1)
        s = np.abs(ref[:, off:off + size]).max(axis=1)
        for f in range(ref.shape[0]):
            if s[f] == 0.0 and d[f] == 0.0:
                continue
            out.append((float(d[f] / max(s[f], floor, 1e-300)), f, name, float(s[f])))
        off += size
    out.sort(key=lambda e: -e[0])
    return out


def magnitude_errors(g, ref, mag, layout, eps, kink=None):
    """Errors of a gradient against its reference, entry by entry, in units
    of the bound eps * mag + kink: mag is the oracle's magnitude of each entry
    (the same sums with every operand taken by absolute value, so |ref| <=
    mag; a rounding of relative size u in every term moves an entry by at
    most u times it per rounding on its longest chain), kink the oracle's
    magnitude of the terms through ReLU units whose pre-activation lies
    within the compared computation's pre-activation error of zero (such a
    unit may take the other branch and add or drop its term whole). One
    (max over the block of |g - ref| / bound, field, tensor name,
    max|ref| / max mag) per (field, tensor) block, worst first; the bound
    holds where every value is at most 1."""
    g = np.atleast_2d(np.asarray(g, np.float64))
    ref = np.atleast_2d(np.asarray(ref, np.float64))
    mag = np.atleast_2d(np.asarray(mag, np.float64))
    kin = np.zeros_like(mag) if kink is None else np.atleast_2d(np.asarray(kink, np.float64))
    out = []
    off = 0
    for name, shape in layout:
        size = int(np.prod(shape))
        sl = slice(off, off + size)
        for f in range(ref.shape[0]):
            m = mag[f, sl]
            bound = eps * m + kin[f, sl]
            d = np.abs(g[f, sl] - ref[f, sl])
            if not m.any():
                assert not d.any(), (f, name)      # untouched blocks are exactly zero
                continue
            err = float(np.max(np.where(bound > 0, d / np.where(bound > 0, bound, 1.0), np.where(d > 0, np.inf, 0.0))))
            out.append((err, f, name, float(np.abs(ref[f, sl]).max() / m.max())))
        off += size
    out.sort(key=lambda e: -e[0])
    return out


def describe(errs, k=3):
    return ", ".join(f"{e:.3g} (field {f} {n}, scale {s:.3g})" for e, f, n, s in errs[:k])


def training_rays(orc, sc, N, W=2048, H=1024, n_cams=20):
    """The first N rays of the training-batch recipe: camera ~ U{0..19},
    pixel ~ U(W x H), equirect rays from the oracle's ray generation."""
    cams = synth.camera_centres(sc, n_cams)
    cam, u, v = synth.ray_draws(N, n_cams, W, H)
    o = np.empty((3, N), np.float32)
    d = np.empty((3, N), np.float32)
    for k in range(n_cams):
        sel = np.nonzero(cam == k)[0]
        if len(sel):
            ok, dk = orc.equirect_rays(W, H, synth.c2w_at(cams[k]), v[sel].astype(np.int64) * W + u[sel])
            o[:, sel] = ok
            d[:, sel] = dk
    return o, d


def training_targets(orc, sc, o, d, batch=65536):
    """Targets of the first N rays of the batch: the teacher field set
    rendered by the oracle plus N(0, 0.01^2) noise, the noise drawn at the
    same counters as for the whole batch (channel c of ray r at c * batch + r)."""
    N = o.shape[1]
    t_rgb, _, _ = orc.render_rays(sc, o, d, weights=synth.teacher_weights(sc))
    idx = (np.arange(3)[:, None] * batch + np.arange(N)[None, :]).astype(np.uint64)
    nz = 0.01 * synth.normal(synth.MASTER_SEED, synth.STREAM_NOISE, idx)
    return (t_rgb + nz).astype(np.float32)
