"""Pins for the FP64 oracle: closed forms, invariants, brute force and
numbers printed in the paper. None of these re-derive a value from the
oracle's own code path; each is chosen so that a dropped term, a wrong sign
or index, or a transposed operand in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# Parameter counts printed in the paper (App. C, Sec. 6.2)
# ---------------------------------------------------------------------------

def test_param_counts_match_paper(orc):
    g = golden("paper_constants.json")
    assert orc.local_params(32) == g["tiny_mlp_params"]["value"]
    assert synth.n_params(synth.local_mlp_layout(32)) == g["tiny_mlp_params"]["value"]
    gp = orc.global_params(256, 128)
    assert abs(gp - g["global_mlp_params_approx"]["value"]) <= g["global_mlp_params_approx"]["rel_tol"] * 596000
    assert gp == synth.n_params(synth.global_mlp_layout())
    n200 = 200 * orc.local_params(32)
    assert abs(n200 - 1.2e6) <= 0.05 * 1.2e6
    assert orc.local_params(64) == 18564


# ---------------------------------------------------------------------------
# Ray generation (Eq.2 / Eq.3)
# ---------------------------------------------------------------------------

def test_equirect_round_trip(orc):
    W, H = 64, 32
    o, d = orc.equirect_rays(W, H, synth.IDENTITY_C2W)
    d64 = d.astype(np.float64)
    phi = np.arctan2(d64[0], d64[2])
    theta = -np.arcsin(np.clip(d64[1], -1, 1))
    u = phi * W / (2 * np.pi) + W / 2 - 0.5          # Eq.2 forward, minus the pixel centre
    v = -theta * H / np.pi + H / 2 - 0.5
    uu, vv = np.meshgrid(np.arange(W), np.arange(H))
    assert np.max(np.abs(u - uu.ravel())) < 1e-3
    assert np.max(np.abs(v - vv.ravel())) < 1e-3
    assert np.all(o == 0)


def test_equirect_special_directions(orc):
    W, H = 256, 128
    o, d = orc.equirect_rays(W, H, synth.IDENTITY_C2W)
    d = d.reshape(3, H, W).astype(np.float64)
    # |d| = 1 to a few FP32 ulp (not renormalised)
    nrm = np.sqrt((d ** 2).sum(0))
    assert np.max(np.abs(nrm - 1)) < 4 * 2.0 ** -24 * 2
    # top row points up (y down): d_y = -sin(theta_0), theta_0 = pi (H - 1) / (2H)
    assert np.allclose(d[1, 0, :], -np.sin(np.pi * (H - 1) / (2 * H)), atol=1e-7)
    assert np.allclose(d[1, H - 1, :], np.sin(np.pi * (H - 1) / (2 * H)), atol=1e-7)
    # the two central columns straddle +z symmetrically
    c0, c1 = W // 2 - 1, W // 2
    assert np.allclose(d[0, :, c0], -d[0, :, c1]) and np.all(d[2, H // 2, c0:c1 + 1] > 0.99)
    # column 0 looks backwards (phi near -pi)
    assert np.all(d[2, H // 2, 0] < -0.99)


def test_pinhole_directions(orc):
    W, H = 64, 48
    f = W / 2.0                                         # 90 degree horizontal field of view
    o, d = orc.pinhole_rays(W, H, f, f, synth.c2w_at((1.0, 2.0, 3.0)))
    d = d.reshape(3, H, W).astype(np.float64)
    assert np.allclose(o[:, 0], [1, 2, 3])
    # right-most column centre: x/z = ((W - 1/2) - W/2)/f
    assert np.allclose(d[0, :, -1] / d[2, :, -1], (W - 0.5 - W / 2) / f, atol=1e-6)
    assert np.allclose(np.sqrt((d ** 2).sum(0)), 1, atol=1e-6)
    # quarter-turn yaw maps +z to +x (rotation entries 0/+-1: exact)
    o2, d2 = orc.pinhole_rays(W, H, f, f, synth.c2w_yaw((0, 0, 0), 1))
    o1, d1 = orc.pinhole_rays(W, H, f, f, synth.c2w_yaw((0, 0, 0), 0))
    assert np.array_equal(d2[0], d1[2]) and np.array_equal(d2[2], -d1[0]) and np.array_equal(d2[1], d1[1])


# ---------------------------------------------------------------------------
# Voxel traversal (FP32 specification) against FP64 brute force
# ---------------------------------------------------------------------------

def brute_segments(scene, o, d, near=0.0, far=np.inf):
    """All positive-length voxel segments by an FP64 slab test per voxel."""
    n, lo, vs = scene.n, scene.lo, scene.voxel
    o = o.astype(np.float64); d = d.astype(np.float64)
    idx = np.arange(n)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    boxes_lo = [lo + i * vs, lo + j * vs, lo + k * vs]
    tin = np.full(i.shape, -np.inf); tout = np.full(i.shape, np.inf)
    for a in range(3):
        blo, bhi = boxes_lo[a], boxes_lo[a] + vs
        if d[a] != 0:
            ta, tb = (blo - o[a]) / d[a], (bhi - o[a]) / d[a]
            tin = np.maximum(tin, np.minimum(ta, tb)); tout = np.minimum(tout, np.maximum(ta, tb))
        else:
            inside = (o[a] >= blo) & (o[a] < bhi)
            tin = np.where(inside, tin, np.inf)
    tin = np.maximum(tin, near); tout = np.minimum(tout, far)
    keep = (tout > tin) & scene.occupied & (scene.field_map >= 0)
    lin = (i + n * (j + n * k))[keep]
    a_in, a_out = tin[keep], tout[keep]
    order = np.argsort(a_in)
    return lin[order], a_in[order], a_out[order], tin, tout


def test_dda_matches_brute_force(orc):
    checked = 0
    for n, seed in ((2, 1), (4, 2), (8, 3)):
        sc = synth.tiny_scene(n, seed, p_occ=0.6, max_samples=64)
        rng = np.random.default_rng(seed)
        N = 300
        o = rng.uniform(-5, 5, size=(3, N)).astype(np.float32)
        d = rng.normal(size=(3, N)); d /= np.linalg.norm(d, axis=0)
        d = d.astype(np.float32)
        smp = orc.sample_rays(sc, o, d)
        for r in range(N):
            lin, tin, tout, all_in, all_out = brute_segments(sc, o[:, r], d[:, r])
            seglen = all_out - all_in
            if np.any((seglen > 0) & (seglen < 1e-4)):
                continue                                   # grazing an edge: tie region
            a, b = smp["offsets"][r], smp["offsets"][r + 1]
            assert np.array_equal(smp["voxel"][a:b], lin), (n, r)
            tm = 0.5 * (tin + tout)
            assert np.allclose(smp["t_mid"][a:b], tm, rtol=0, atol=4e-6 * max(1.0, np.max(np.abs(tm), initial=1)))
            assert np.allclose(smp["delta"][a:b], tout - tin, rtol=0, atol=4e-6 * max(1.0, np.max(np.abs(tm), initial=1)))
            assert np.all(smp["ray_id"][a:b] == r)
            assert np.array_equal(smp["field"][a:b], sc.field_map.ravel()[lin])
            checked += 1
    assert checked > 700


def test_dda_axis_aligned_full_voxels(orc):
    sc = synth.tiny_scene(8, 5, p_occ=1.0)
    o = np.array([[-3.9], [0.1], [0.2]], np.float32)
    d = np.array([[1.0], [0.0], [0.0]], np.float32)
    smp = orc.sample_rays(sc, o, d)
    assert smp["counts"][0] == 8
    # every full voxel has delta exactly one voxel edge; the first is partial
    assert np.all(smp["delta"][1:] == np.float32(1.0))
    assert smp["delta"][0] == np.float32(-3.0) - np.float32(-3.9)
    assert list(smp["voxel"]) == [i + 8 * (4 + 8 * 4) for i in range(8)]


def test_dda_full_grid_lengths_telescope(orc):
    sc = synth.tiny_scene(8, 6, p_occ=1.0, max_samples=64)
    rng = np.random.default_rng(7)
    N = 200
    o = rng.uniform(-3, 3, size=(3, N)).astype(np.float32)
    d = rng.normal(size=(3, N)); d /= np.linalg.norm(d, axis=0); d = d.astype(np.float32)
    smp = orc.sample_rays(sc, o, d)
    for r in range(N):
        t1 = np.min(np.maximum((-4 - o[:, r].astype(np.float64)) / d[:, r], (4 - o[:, r].astype(np.float64)) / d[:, r]))
        a, b = smp["offsets"][r], smp["offsets"][r + 1]
        assert abs(smp["delta"][a:b].astype(np.float64).sum() - t1) < 1e-5


def test_dda_corner_start_diagonal_tie(orc):
    # camera exactly on the centre corner of an 8^3 grid of 1 m voxels, moving
    # along the (-1,-1,-1) diagonal: only the diagonal voxels have positive
    # length; ties across planes emit nothing.
    sc = synth.tiny_scene(8, 8, p_occ=1.0)
    o = np.zeros((3, 1), np.float32)
    s = np.float32(-1 / np.sqrt(3))
    d = np.array([[s], [s], [s]], np.float32)
    smp = orc.sample_rays(sc, o, d)
    assert [int(v) for v in smp["voxel"]] == [c + 8 * (c + 8 * c) for c in (3, 2, 1, 0)]
    assert np.allclose(smp["delta"], np.sqrt(3), rtol=1e-6)
    # the same along +x from the corner: voxel row (4.., 4, 4) -- floor picks the upper voxel
    d = np.array([[1.0], [0.0], [0.0]], np.float32)
    smp = orc.sample_rays(sc, o, d)
    assert [int(v) for v in smp["voxel"]] == [i + 8 * (4 + 8 * 4) for i in range(4, 8)]
    # and along -x: the lower voxel on the start plane
    d = np.array([[-1.0], [0.0], [0.0]], np.float32)
    smp = orc.sample_rays(sc, o, d)
    assert [int(v) for v in smp["voxel"]] == [i + 8 * (4 + 8 * 4) for i in (3, 2, 1, 0)]


def test_dda_near_far_and_cap(orc):
    sc = synth.tiny_scene(8, 9, p_occ=0.7, max_samples=64)
    rng = np.random.default_rng(10)
    N = 100
    o = rng.uniform(-2, 2, size=(3, N)).astype(np.float32)
    d = rng.normal(size=(3, N)); d /= np.linalg.norm(d, axis=0); d = d.astype(np.float32)
    full = orc.sample_rays(sc, o, d)
    capped = orc.sample_rays(sc, o, d, max_samples=3)
    clipped = orc.sample_rays(sc, o, d, near=1.0, far=3.0)
    for r in range(N):
        a, b = full["offsets"][r], full["offsets"][r + 1]
        ca, cb = capped["offsets"][r], capped["offsets"][r + 1]
        assert cb - ca == min(3, b - a)
        assert np.array_equal(capped["voxel"][ca:cb], full["voxel"][a:a + (cb - ca)])
        ka, kb = clipped["offsets"][r], clipped["offsets"][r + 1]
        tm, dl = clipped["t_mid"][ka:kb], clipped["delta"][ka:kb]
        assert np.all(tm - dl / 2 >= 1.0 - 1e-6) and np.all(tm + dl / 2 <= 3.0 + 1e-6)


def test_dda_counts_on_small_config(orc):
    # strictly increasing t, positive deltas, segments do not overlap
    sc = synth.scene_small()
    o, d = orc.equirect_rays(256, 128, synth.IDENTITY_C2W)
    smp = orc.sample_rays(sc, o, d)
    assert smp["counts"].max() <= 32 and np.all(smp["delta"] > 0)
    ends = smp["t_mid"] + smp["delta"] / 2
    starts = smp["t_mid"] - smp["delta"] / 2
    same = smp["ray_id"][1:] == smp["ray_id"][:-1]
    assert np.all(starts[1:][same] >= ends[:-1][same] - 1e-6)
    assert np.all(sc.occupied.ravel()[smp["voxel"]])


# ---------------------------------------------------------------------------
# Positional encoding
# ---------------------------------------------------------------------------

def test_encoding_layout_and_closed_values(orc):
    assert len(orc.encode([0.1, 0.2, 0.3], 10)) == 63 and len(orc.encode([0.1, 0.2, 0.3], 4)) == 27
    g = orc.encode([0.0, 0.5, 1.0], 10)
    assert list(g[:3]) == [0.0, 0.5, 1.0]
    for l in range(10):
        s, c = g[3 + 6 * l: 6 + 6 * l], g[6 + 6 * l: 9 + 6 * l]
        # x = 0: sin 0, cos 1
        assert s[0] == 0.0 and c[0] == 1.0
        # x = 1/2: sin(2^l pi / 2) and cos(2^l pi / 2)
        assert s[1] == (1.0 if l == 0 else 0.0)
        assert c[1] == (0.0 if l == 0 else (-1.0 if l == 1 else 1.0))
        # x = 1: sin(2^l pi) = 0, cos = -1 for l = 0 else 1
        assert s[2] == 0.0 and c[2] == (-1.0 if l == 0 else 1.0)


def test_encoding_unit_circle_and_frequency(orc):
    rng = np.random.default_rng(0)
    for _ in range(50):
        x = rng.uniform(-1.3, 1.3, 3)
        g = orc.encode(x, 10)
        for l in range(10):
            s, c = g[3 + 6 * l: 6 + 6 * l], g[6 + 6 * l: 9 + 6 * l]
            assert np.allclose(s ** 2 + c ** 2, 1.0, atol=1e-14)
            assert np.allclose(s, np.sin(np.pi * 2.0 ** l * x), atol=1e-12)
            assert np.allclose(c, np.cos(np.pi * 2.0 ** l * x), atol=1e-12)


# ---------------------------------------------------------------------------
# Local MLP
# ---------------------------------------------------------------------------

def _zeros_local(h):
    lay = synth.local_mlp_layout(h)
    w = np.zeros(synth.n_params(lay), np.float32)
    return lay, w, synth.unpack(lay, w)


def sp(z):
    return max(z, 0) + math.log1p(math.exp(-abs(z)))


def sg(z):
    return 1 / (1 + math.exp(-z))


def test_local_mlp_zero_weights(orc):
    lay, w, t = _zeros_local(32)
    t["bs"][0] = 0.37
    t["b4"][:] = [-0.5, 0.25, 1.5]
    t["b1"][:] = 3.0; t["b2"][:] = -1.0; t["b3"][:] = 2.0
    sigma, rgb = orc.local_mlp(w, 32, [0.1, -0.2, 0.3], [0, 0, 1])
    assert abs(sigma - sp(float(np.float32(0.37)))) < 1e-15
    assert np.allclose(rgb, [sg(-0.5), sg(0.25), sg(1.5)], atol=1e-15)


def test_local_mlp_routed_signal(orc):
    """Hand-wired weights carry known signals through distinct indices of
    every layer; a transposed matrix, a wrong offset or a wrong encoding
    slot moves the signal and changes the closed-form result."""
    h = 32
    lay, w, t = _zeros_local(h)
    x, y, z = 0.3, 0.1, 0.05
    dvec = np.array([0.6, 0.0, 0.8])
    # density path: raw x -> h1[5] -> h2[7] (x2) -> sigma
    t["W1"][5, 0] = 1.0
    t["W2"][7, 5] = 2.0
    t["ws"][0, 7] = 1.5; t["bs"][0] = -0.25
    # colour path: sin(4 pi y) (l=2, sine, component y) -> h1[2] -> h2[9] -> f[12] -> h3[6] -> red
    t["W1"][2, 3 + 6 * 2 + 1] = 1.0
    t["W2"][9, 2] = 1.0
    t["Wf"][12, 9] = 1.0
    t["W3"][6, 12] = 1.0
    t["W4"][0, 6] = 1.0
    # cos(4 pi z) -> h1[4] -> h2[10] -> f[13] -> h3[8], plus 0.5 cos(2 pi d_x) -> green
    t["W1"][4, 3 + 6 * 2 + 3 + 2] = 1.0
    t["W2"][10, 4] = 1.0
    t["Wf"][13, 10] = 1.0; t["bf"][13] = 0.125
    t["W3"][8, 13] = 1.0
    t["W3"][8, h + 3 + 6 * 1 + 3 + 0] = 0.5
    t["W4"][1, 8] = 1.0
    # f[12] also reaches blue with a negative sign through h3[3] and the raw direction d_z
    t["W3"][3, 12] = 1.0; t["W3"][3, h + 2] = -2.0; t["b3"][3] = 2.0
    t["W4"][2, 3] = -1.0; t["b4"][2] = 0.5
    sigma, rgb = orc.local_mlp(w, h, [x, y, z], dvec)
    assert abs(sigma - sp(3 * x - 0.25)) < 1e-14
    f12 = max(math.sin(4 * math.pi * y), 0)
    assert abs(rgb[0] - sg(f12)) < 1e-14
    h38 = max(max(math.cos(4 * math.pi * z), 0) + 0.125 + 0.5 * math.cos(2 * math.pi * 0.6), 0)
    assert abs(rgb[1] - sg(h38)) < 1e-14
    h33 = max(f12 - 2 * 0.8 + 2.0, 0)
    assert abs(rgb[2] - sg(0.5 - h33)) < 1e-14


def test_local_mlp_feature_is_linear(orc):
    """The tiny network's feature layer has no activation (App. C, tiny-network
    table): a negative feature must reach the colour layer with its sign, and a
    feature that is negative only through its bias must still add its value."""
    h = 32
    lay, w, t = _zeros_local(h)
    x = 0.3
    t["W1"][5, 0] = 1.0                        # raw x -> h1[5] = x
    t["W2"][7, 5] = 1.0                        # -> h2[7] = x
    t["Wf"][20, 7] = -1.0; t["bf"][20] = -0.25  # f[20] = -x - 0.25 < 0
    t["W3"][6, 20] = -1.0                      # h3[6] = relu(x + 0.25)
    t["W4"][0, 6] = 1.0
    t["Wf"][21, 7] = 1.0; t["bf"][21] = -0.75  # f[21] = x - 0.75 = -0.45
    t["W3"][8, 21] = 1.0; t["b3"][8] = 1.0     # h3[8] = relu(1 + f[21]) = 0.55
    t["W4"][1, 8] = 2.0; t["b4"][1] = -1.0
    sigma, rgb = orc.local_mlp(w, h, [x, 0.1, 0.05], [0.6, 0.0, 0.8])
    assert abs(rgb[0] - sg(x + 0.25)) < 1e-14
    assert abs(rgb[1] - sg(2 * (1.0 + x - 0.75) - 1.0)) < 1e-14


def test_local_mlp_single_layer_against_matmul(orc):
    """With identity-like downstream layers the red output is sigmoid of one
    ReLU dense layer of the encoding, checked against numpy's matmul."""
    h = 32
    lay, w, t = _zeros_local(h)
    rng = np.random.default_rng(3)
    t["W1"][:] = rng.normal(size=t["W1"].shape).astype(np.float32) * 0.2
    t["b1"][:] = rng.normal(size=h).astype(np.float32) * 0.1
    for k in range(h):
        t["W2"][k, k] = 1.0
    t["Wf"][0, :] = 1.0 / h
    t["W3"][0, 0] = 1.0
    t["W4"][0, 0] = 1.0
    xh = np.array([0.21, -0.43, 0.77])
    sigma, rgb = orc.local_mlp(w, h, xh, [0, 1, 0])
    # encoding by its definition, via numpy
    enc = [*xh]
    for l in range(10):
        enc += list(np.sin(np.pi * 2.0 ** l * xh)) + list(np.cos(np.pi * 2.0 ** l * xh))
    h1 = np.maximum(t["W1"].astype(np.float64) @ np.array(enc) + t["b1"], 0)
    assert abs(rgb[0] - sg(max(h1.mean(), 0))) < 1e-12


# ---------------------------------------------------------------------------
# Compositing (Eq.4 / Eq.5)
# ---------------------------------------------------------------------------

def test_composite_constant_density_closed_form(orc):
    sigma0, n, L, t0 = 1.7, 13, 2.3, 0.4
    dl = L / n
    tm = t0 + (np.arange(n) + 0.5) * dl
    col = np.tile([0.2, 0.5, 0.9], (n, 1))
    C, D, A, w = orc.composite(np.full(n, sigma0), col, tm, np.full(n, dl))
    assert abs(A - (1 - math.exp(-sigma0 * L))) < 1e-14
    assert abs(w.sum() - A) < 1e-15
    assert np.allclose(C, np.array([0.2, 0.5, 0.9]) * A, atol=1e-15)
    r = math.exp(-sigma0 * dl)
    Dc = (1 - r) * ((t0 + dl / 2) * (1 - r ** n) / (1 - r) + dl * (r - n * r ** n + (n - 1) * r ** (n + 1)) / (1 - r) ** 2)
    assert abs(D - Dc) < 1e-13


def test_composite_special_cases(orc):
    C, D, A, w = orc.composite([0.8], [[0.1, 0.2, 0.3]], [2.0], [0.5])
    a = 1 - math.exp(-0.4)
    assert abs(A - a) < 1e-15 and abs(D - 2.0 * a) < 1e-15 and np.allclose(C, np.array([0.1, 0.2, 0.3]) * a)
    C, D, A, w = orc.composite(np.zeros(5), np.ones((5, 3)), np.arange(5.0), np.ones(5))
    assert A == 0 and D == 0 and np.all(C == 0)
    C, D, A, w = orc.composite([], np.zeros((0, 3)), [], [])
    assert A == 0
    # an opaque first sample hides everything behind it; order matters
    C, D, A, w = orc.composite([50.0, 1.0], [[1, 0, 0], [0, 1, 0]], [1.0, 2.0], [1.0, 1.0])
    assert w[0] == 1 - math.exp(-50.0) and w[1] < 1e-20 and C[1] < 1e-20
    rng = np.random.default_rng(1)
    s = rng.uniform(0, 3, 40); dl = rng.uniform(0.01, 0.2, 40)
    C, D, A, w = orc.composite(s, rng.uniform(0, 1, (40, 3)), np.cumsum(dl), dl)
    T_final = math.exp(-(s * dl).sum())
    assert abs(A - (1 - T_final)) < 1e-14 and A <= 1


def test_composite_backward_finite_difference(orc):
    rng = np.random.default_rng(2)
    n = 9
    s = rng.uniform(0.1, 4, n); col = rng.uniform(0, 1, (n, 3)); dl = rng.uniform(0.05, 0.4, n)
    tm = np.cumsum(dl)
    g = rng.normal(size=3)
    ds, dc = orc.composite_backward(s, col, dl, g)

    def L(s_, c_):
        C, _, _, _ = orc.composite(s_, c_, tm, dl)
        return float(C @ g)
    for i in range(n):
        e = 1e-6
        sp_, sm_ = s.copy(), s.copy(); sp_[i] += e; sm_[i] -= e
        assert abs((L(sp_, col) - L(sm_, col)) / (2 * e) - ds[i]) < 1e-8
        for c in range(3):
            cp, cm = col.copy(), col.copy(); cp[i, c] += e; cm[i, c] -= e
            assert abs((L(s, cp) - L(s, cm)) / (2 * e) - dc[i, c]) < 1e-8
    # one sample: dC/dsigma = delta exp(-sigma delta) c
    ds1, _ = orc.composite_backward([0.7], [[0.3, 0.6, 0.9]], [0.25], [1.0, 0.0, 0.0])
    assert abs(ds1[0] - 0.25 * math.exp(-0.7 * 0.25) * 0.3) < 1e-15


# ---------------------------------------------------------------------------
# Whole local path: batched oracle vs per-sample evaluation + naive compositing
# ---------------------------------------------------------------------------

def test_render_equals_per_sample_evaluation(orc):
    sc = synth.tiny_scene(8, 11, p_occ=0.4, n_fields=3, hidden=32)
    rng = np.random.default_rng(11)
    N = 40
    o = rng.uniform(-3, 3, size=(3, N)).astype(np.float32)
    d = rng.normal(size=(3, N)); d /= np.linalg.norm(d, axis=0); d = d.astype(np.float32)
    rgb, depth, opac = orc.render_rays(sc, o, d)
    smp = orc.sample_rays(sc, o, d)
    sig_b, rgb_b = orc.sample_outputs(sc, o, d, smp["offsets"])
    P = sc.n_params
    for r in range(N):
        a, b = smp["offsets"][r], smp["offsets"][r + 1]
        sig, col = [], []
        for j in range(a, b):
            # encoding input by the FP32 specification: p = fma(t, d, o), xhat = p / 4
            p = np.array([np.float32(np.float64(smp["t_mid"][j]) * np.float64(d[k, r]) + np.float64(o[k, r]))
                          for k in range(3)], np.float32)
            s1, c1 = orc.local_mlp(sc.weights[smp["field"][j]], 32, (p * np.float32(0.25)).astype(np.float64),
                                   d[:, r].astype(np.float64))
            sig.append(s1); col.append(c1)
            assert abs(s1 - sig_b[j]) < 1e-12 and np.allclose(c1, rgb_b[:, j], atol=1e-12)
        C, D, A, _ = orc.composite(sig, np.array(col).reshape(-1, 3), smp["t_mid"][a:b], smp["delta"][a:b])
        assert np.allclose(C, rgb[:, r], atol=1e-12) and abs(D - depth[r]) < 1e-11 and abs(A - opac[r]) < 1e-12


# ---------------------------------------------------------------------------
# Loss gradient of the local path: analytic vs central finite differences
# ---------------------------------------------------------------------------

def _fd_check(loss_fn, w, idx, grad, rel=1e-5):
    bad = []
    for i in idx:
        base = w[i]
        hstep = np.float32(max(abs(base), 1e-2) * 2e-4)
        wp, wm = w.copy(), w.copy()
        wp[i] = base + hstep; wm[i] = base - hstep
        eff = np.float64(wp[i]) - np.float64(wm[i])
        fd = (loss_fn(wp) - loss_fn(wm)) / eff
        wp2, wm2 = w.copy(), w.copy()
        wp2[i] = base + hstep / 2; wm2[i] = base - hstep / 2
        fd2 = (loss_fn(wp2) - loss_fn(wm2)) / (np.float64(wp2[i]) - np.float64(wm2[i]))
        if abs(fd - fd2) > 1e-3 * max(abs(fd), 1e-9):
            continue                                   # a ReLU kink inside the stencil
        if abs(fd - grad[i]) > rel * max(abs(fd), 1e-7) + 1e-12:
            bad.append((i, fd, grad[i]))
    return bad


def test_train_grad_finite_difference(orc):
    sc = synth.tiny_scene(4, 12, p_occ=0.5, n_fields=2, hidden=16)
    rng = np.random.default_rng(12)
    N = 12
    o = rng.uniform(-1, 1, size=(3, N)).astype(np.float32)
    d = rng.normal(size=(3, N)); d /= np.linalg.norm(d, axis=0); d = d.astype(np.float32)
    # give the fields some non-zero biases so that every layer carries gradient
    w0 = sc.weights.copy()
    w0 += rng.normal(size=w0.shape).astype(np.float32) * 0.05
    target = rng.uniform(0, 1, (3, N)).astype(np.float32)
    loss, grad, _ = orc.train_grad(sc, o, d, target, weights=w0)
    flat = w0.ravel()

    def loss_fn(wf):
        l, _, _ = orc.train_grad(sc, o, d, target, weights=wf.reshape(w0.shape))
        return l
    idx = rng.choice(flat.size, 150, replace=False)
    # include every bias group and the density head explicitly
    lay = synth.local_mlp_layout(16)
    off = 0
    for name, shape in lay:
        size = int(np.prod(shape))
        idx = np.append(idx, [off, off + size - 1])
        off += size
    bad = _fd_check(loss_fn, flat, idx, grad.ravel())
    assert not bad, bad[:5]
    assert np.count_nonzero(grad) > 0.3 * grad.size


def test_train_grad_magnitude_bounds_the_gradient(orc):
    """The magnitude of each gradient entry (every operand of the forward and
    backward taken by absolute value) bounds the entry by the triangle
    inequality, is not changed by asking for it, and equals the entry where
    all its terms are non-negative: with zero weight matrices, positive
    biases and zero targets, dL/dC = 2C/(3B) >= 0, the colour layer sees
    h3 = relu(b3) >= 0, so the W4 and b4 gradients are sums of non-negative
    terms and their magnitudes are the gradients themselves."""
    sc = synth.tiny_scene(6, 31, p_occ=0.5, n_fields=3, hidden=16, max_samples=20)
    rng = np.random.default_rng(31)
    N = 200
    o = rng.uniform(-2, 2, size=(3, N)).astype(np.float32)
    d = rng.normal(size=(3, N)); d /= np.linalg.norm(d, axis=0); d = d.astype(np.float32)
    w0 = (sc.weights + rng.normal(size=sc.weights.shape).astype(np.float32) * 0.05).astype(np.float32)
    target = rng.uniform(0, 1, (3, N)).astype(np.float32)
    loss, grad, rgb = orc.train_grad(sc, o, d, target, weights=w0)
    loss_m, grad_m, rgb_m, mag = orc.train_grad(sc, o, d, target, weights=w0, magnitude=True)
    assert loss_m == loss and np.array_equal(grad_m, grad) and np.array_equal(rgb_m, rgb)
    assert np.all(mag >= np.abs(grad) * (1 - 1e-12))
    assert np.all(mag[grad != 0] > 0)
    # cancellation is visible: some entries are far below their magnitude
    ratio = np.abs(grad[mag > 0]) / mag[mag > 0]
    assert ratio.min() < 1e-2 and np.median(ratio) > 1e-4

    lay = synth.local_mlp_layout(16)
    wz = np.zeros_like(w0)
    off = {}
    o_ = 0
    for name, shape in lay:
        size = int(np.prod(shape))
        off[name] = (o_, o_ + size)
        if len(shape) == 1:   # biases
            wz[:, o_:o_ + size] = rng.uniform(0.1, 0.5, (sc.n_fields, size))
        o_ += size
    _, gz, _, mz = orc.train_grad(sc, o, d, np.zeros((3, N), np.float32), weights=wz, magnitude=True)
    for name in ("W4", "b4"):
        a, b = off[name]
        assert np.any(gz[:, a:b] > 0)
        assert np.array_equal(mz[:, a:b], gz[:, a:b]), name
    a, b = off["bs"]
    assert np.all(mz[:, a:b] >= np.abs(gz[:, a:b]))
    # kink terms: none at tau = 0 (no pre-activation is exactly zero here),
    # more with a wider band, and at most the magnitude itself
    _, _, _, m0, k0 = orc.train_grad(sc, o, d, target, weights=w0, magnitude=True, kink=0.0)
    _, _, _, m1, k1 = orc.train_grad(sc, o, d, target, weights=w0, magnitude=True, kink=1e-2)
    _, _, _, m2, k2 = orc.train_grad(sc, o, d, target, weights=w0, magnitude=True, kink=1e9)
    assert np.array_equal(m0, mag) and np.array_equal(m1, mag)
    assert not k0.any() and np.all(k1 >= 0) and np.any(k1 > 0) and np.all(k2 >= k1)
    # with every unit in the band, the kink terms contain every term that
    # passes a ReLU unit (W1..W3, Wf and their biases reach the loss through
    # one; inactive units and paths through several units add more), and
    # none of the heads that pass none (W4, b4 and the density head)
    for name in ("W1", "b1", "W2", "b2", "Wf", "bf", "W3", "b3"):
        a, b = off[name]
        assert np.all(k2[:, a:b] >= mag[:, a:b] * (1 - 1e-12)) and np.any(k2[:, a:b] > mag[:, a:b]), name
    for name in ("W4", "b4", "ws", "bs"):
        a, b = off[name]
        assert not k2[:, a:b].any(), name


# ---------------------------------------------------------------------------
# Global omnidirectional field
# ---------------------------------------------------------------------------

def test_invdepth_samples(orc):
    t, dl = orc.invdepth_t(128, 0.1, 20.0)
    assert abs(t[0] - 0.1) < 1e-7 and abs(t[-1] - 20.0) < 4e-6
    inv = 1.0 / t.astype(np.float64)
    assert np.allclose(np.diff(inv), (1 / 20.0 - 1 / 0.1) / 127, rtol=1e-4)
    assert np.all(np.diff(t) > 0) and dl[-1] == 0 and np.allclose(dl[:-1], np.diff(t))


def test_global_mlp_zero_weights_and_skip(orc):
    lay = synth.global_mlp_layout(16, color_width=8)
    w = np.zeros(synth.n_params(lay), np.float32)
    t = synth.unpack(lay, w)
    t["bs"][0] = 0.5; t["b11"][:] = [0.1, -0.2, 0.3]
    s, rgb = orc.global_mlp(w, [0.1, 0.2, 0.3], [0, 0, 1], width=16, color_width=8)
    assert s == 0.5 and np.allclose(rgb, [sg(float(np.float32(v))) for v in (0.1, -0.2, 0.3)], atol=1e-15)
    # the skip: encoded position re-enters at the fifth layer (its slot 16 + 2 = raw z)
    t["W5"][3, 16 + 2] = 1.0
    t["W6"][3, 3] = 1.0; t["W7"][3, 3] = 1.0; t["W8"][3, 3] = 1.0
    t["ws"][0, 3] = 2.0
    s, _ = orc.global_mlp(w, [0.1, 0.2, 0.3], [0, 0, 1], width=16, color_width=8)
    assert abs(s - (0.5 + 2 * 0.3)) < 1e-15
    # the layer-8 output has no activation: a negative value passes through to sigma's ReLU input
    t["bs"][0] = 0.0; t["b8"][3] = -1.0
    s, _ = orc.global_mlp(w, [0.1, 0.2, 0.3], [0, 0, 1], width=16, color_width=8)
    assert abs(s - max(2 * (0.3 - 1.0), 0)) < 1e-15
    t["ws"][0, 3] = -2.0
    s, _ = orc.global_mlp(w, [0.1, 0.2, 0.3], [0, 0, 1], width=16, color_width=8)
    assert abs(s - 1.4) < 1e-15


def test_global_mlp_colour_branch_routed(orc):
    """The 360NeRF table's colour branch: f = ReLU(Wf h8 + bf), then layer 10
    on [f ; gamma(d)] with a ReLU, then sigmoid. A raw coordinate is carried
    through the trunk to h8 and then split into signals that only the right
    activations and the right input order reproduce in closed form."""
    width, cw, dd = 16, 8, 27
    lay = synth.global_mlp_layout(width, color_width=cw)
    w = np.zeros(synth.n_params(lay), np.float32)
    t = synth.unpack(lay, w)
    x = 0.3
    d = np.array([0.48, 0.6, 0.64])              # unit length
    t["W1"][3, 0] = 1.0                          # raw x -> h1[3] = x
    for k in (2, 3, 4, 5, 6, 7, 8):
        t[f"W{k}"][3, 3] = 1.0                   # the h part of layer 5's [h4 ; gx] input comes first
    # feature ReLU: f5 = relu(-x) = 0, f6 = relu(x) = x; layer 10 row 2 adds both
    t["Wf"][5, 3] = -1.0; t["Wf"][6, 3] = 1.0
    t["W10"][2, 5] = 1.0; t["W10"][2, 6] = 1.0
    t["W11"][0, 2] = 1.0
    # layer 10 ReLU: row 4 = relu(-f6) = 0 feeds green beside a bias
    t["W10"][4, 6] = -1.0
    t["W11"][1, 4] = 1.0; t["b11"][1] = 0.25
    # gamma(d) follows f in layer 10's input: sin(2 pi d_y) (l = 1, y) and raw d_z
    t["W10"][7, width + 3 + 6 * 1 + 1] = 1.0
    t["W10"][7, width + 2] = -0.5
    t["b10"][7] = 1.0
    t["W11"][2, 7] = 1.0
    s, rgb = orc.global_mlp(w, [x, 0.2, 0.1], d, width=width, color_width=cw)
    assert s == 0.0
    assert abs(rgb[0] - sg(x)) < 1e-14
    assert abs(rgb[1] - sg(0.25)) < 1e-14
    h107 = 1.0 + math.sin(2 * math.pi * 0.6) - 0.5 * 0.64
    assert h107 > 0
    assert abs(rgb[2] - sg(h107)) < 1e-14
    # a negative layer-10 pre-activation is clipped, a positive one is not
    t["b10"][7] = -1.0
    s, rgb = orc.global_mlp(w, [x, 0.2, 0.1], d, width=width, color_width=cw)
    assert abs(rgb[2] - 0.5) < 1e-15


def test_global_step_finite_difference_and_occupancy(orc):
    width, cw = 16, 8
    lay = synth.global_mlp_layout(width, color_width=cw)
    rng = np.random.default_rng(13)
    w = synth.xavier_weights(lay, 1, 13, synth.STREAM_WEIGHTS)[0]
    w += rng.normal(size=w.shape).astype(np.float32) * 0.05
    N, ns = 3, 16
    o = rng.uniform(-1, 1, size=(3, N)).astype(np.float32)
    d = rng.normal(size=(3, N)); d /= np.linalg.norm(d, axis=0); d = d.astype(np.float32)
    target = rng.uniform(0, 1, (3, N)).astype(np.float32)
    kw = dict(n_samples=ns, width=width, color_width=cw, grid_n=8, voxel=1.0)
    res = orc.global_step(w, o, d, target, **kw)

    def loss_fn(wf):
        return orc.global_step(wf, o, d, target, occupancy=False, **kw)["loss"]
    idx = rng.choice(w.size, 120, replace=False)
    bad = _fd_check(loss_fn, w, idx, res["grad"])
    assert not bad, bad[:5]
    # occupancy: max of per-sample density over the samples in each voxel,
    # recomputed one sample at a time and independent of visiting order
    t, dl = orc.invdepth_t(ns, 0.1, 20.0)
    occ = np.zeros((8, 8, 8))
    order = rng.permutation(N * ns)
    for q in order:
        r, k = divmod(int(q), ns)
        p = np.array([np.float32(np.float64(t[k]) * d[a, r] + o[a, r]) for a in range(3)], np.float32)
        s1, _ = orc.global_mlp(w, (p * np.float32(0.25)).astype(np.float64), d[:, r].astype(np.float64),
                               width=width, color_width=cw)
        qv = (p.astype(np.float32) - np.float32(-4.0)) * np.float32(1.0)
        if np.all((qv >= 0) & (qv < 8)):
            i = np.floor(qv).astype(int)
            occ[i[2], i[1], i[0]] = max(occ[i[2], i[1], i[0]], s1)
    assert np.allclose(occ, res["occ_max"], atol=1e-12)


# ---------------------------------------------------------------------------
# Adam (Sec. 6.3)
# ---------------------------------------------------------------------------

def test_adam_first_step_is_signed_lr(orc):
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w = np.ones(4); m = np.zeros(4); v = np.zeros(4)
    orc.adam(w, g, m, v, 1, 1e-3)
    assert np.allclose(w, 1 - 1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), atol=1e-15)
    # second step with the same gradient keeps the same magnitude (bias correction)
    orc.adam(w, g, m, v, 2, 1e-3)
    assert np.allclose(w[:3], 1 - 2e-3 * np.sign(g[:3]), atol=1e-9)


# ---------------------------------------------------------------------------
# Stage I probabilistic occupancy (Sec. 4.1, Eq.6, Alg.1)
# ---------------------------------------------------------------------------

def _sig(l):
    return 1.0 / (1.0 + math.exp(-l))


def test_occupancy_logit_range_matches_paper(orc):
    g = golden("paper_constants.json")["logit_range"]
    assert round(_sig(g["hi"]), 2) == g["p_hi"] and round(_sig(g["lo"]), 2) == g["p_lo"]
    assert abs(orc.logit(0.97) - 3.476) < 5e-4 and abs(orc.logit(0.12) - (-1.992)) < 5e-4
    desc = orc.occ_desc(8, -4.0, 1.0)
    o = np.array([[-3.9], [0.5], [0.5]], np.float32)
    d = np.array([[1.0], [0.0], [0.0]], np.float32)
    one = lambda v: np.array([v], np.float32)
    L = np.zeros((8, 8, 8), np.float32)
    # repeated sharp hits (one pose each) saturate at the upper bound; the
    # voxel counts as occupied (p > 0.97) from the first pose whose sum
    # passes logit(0.97): ceil(3.476 / logit(0.7)) = 5
    first = None
    for k in range(1, 9):
        p = orc.occupancy_update(desc, L, o, d, one(4.4), one(0.0), one(1.0))
        if first is None and p[4, 4, 4] > g["p_hi"]:
            first = k
    assert first == math.ceil(math.log(0.97 / 0.03) / math.log(0.7 / 0.3)) == 5
    assert L[4, 4, 4] == np.float32(g["hi"]) and round(float(p[4, 4, 4]), 2) == g["p_hi"]
    # the free voxels in front saturate at the lower bound
    assert np.all(L[4, 4, :4] == np.float32(g["lo"])) and np.all(np.round(p[4, 4, :4], 2) == g["p_lo"])
    assert np.all(L[4, 4, 5:] == 0) and np.count_nonzero(L) == 5


def test_depth_stats_closed_forms(orc):
    t = np.array([[1.0, 2.0, 3.0, 4.0]], np.float32)
    dl = np.array([[1.0, 1.0, 1.0, 0.0]], np.float32)
    # an opaque third sample takes all the weight
    D, U, A = orc.depth_stats(t, dl, np.array([[0, 0, 1e4, 0]], np.float32))
    assert abs(D[0] - 3.0) < 1e-12 and U[0] < 1e-6 and abs(A[0] - 1.0) < 1e-12
    # tau_0 = ln 2 gives w_0 = 1/2; an opaque second sample takes the other half
    D, U, A = orc.depth_stats(t, dl, np.array([[math.log(2.0), 1e4, 0, 0]], np.float32))
    assert abs(A[0] - 1.0) < 1e-7 and abs(D[0] - 1.5) < 1e-7 and abs(U[0] - 0.5) < 1e-7
    # half opacity: normalised weights put the depth at the sample itself
    D, U, A = orc.depth_stats(t[:, :1], dl[:, :1], np.array([[math.log(2.0)]], np.float32))
    assert abs(A[0] - 0.5) < 1e-7 and abs(D[0] - 1.0) < 1e-12 and U[0] == 0.0
    # nothing visible: zero depth and spread
    D, U, A = orc.depth_stats(t, dl, np.zeros((1, 4), np.float32))
    assert D[0] == 0 and U[0] == 0 and A[0] == 0
    # constant density on evenly spaced samples: the weights are geometric,
    # P(i) = (1 - q) q^i with q = exp(-tau), so D = t_0 + dt q / (1 - q) and
    # U = dt sqrt(q) / (1 - q) (the mean and spread of that distribution)
    n, t0, dt, tau = 400, 0.5, 0.125, 0.25
    tt = (t0 + dt * np.arange(n)).astype(np.float32)[None]
    D, U, A = orc.depth_stats(tt, np.full((1, n), dt, np.float32), np.full((1, n), tau / dt, np.float32))
    q = math.exp(-tau)
    assert abs(A[0] - 1.0) < 1e-12
    assert abs(D[0] - (t0 + dt * q / (1 - q))) < 1e-9
    assert abs(U[0] - dt * math.sqrt(q) / (1 - q)) < 1e-9


def test_occupancy_axis_ray_band_and_confidence(orc):
    desc = orc.occ_desc(8, -4.0, 1.0)
    lh, lm = np.float32(orc.logit(0.7)), np.float32(orc.logit(0.4))
    o = np.array([[-3.9], [0.5], [0.5]], np.float32)
    d = np.array([[1.0], [0.0], [0.0]], np.float32)
    one = lambda v: np.array([v], np.float32)

    def row(D, U, A=1.0, oo=o, dd=d):
        L = np.zeros((8, 8, 8), np.float32)
        orc.occupancy_update(desc, L, oo, dd, one(D), one(U), one(A))
        return L

    # sharp depth at x = 0.5 (voxel 4): voxels 0..3 free, 4 hit, the rest untouched
    L = row(4.4, 0.0)
    assert np.array_equal(L[4, 4], np.array([lm] * 4 + [lh, 0, 0, 0], np.float32))
    assert np.count_nonzero(L) == 5
    # uncertainty 1.6 (1.6 voxels): free only up to D - U = 2.8 (voxels 0, 1);
    # 2 and 3 lie in the band; the hit logit is l_hit / (1 + 1.6)
    L = row(4.4, 1.6)
    h = np.float32(lh / (np.float32(1.0) + np.float32(1.6)))
    assert np.array_equal(L[4, 4], np.array([lm, lm, 0, 0, h, 0, 0, 0], np.float32))
    # below the opacity floor: no measurement
    assert np.count_nonzero(row(4.4, 0.0, A=0.4)) == 0
    # a surface beyond the box: every crossed voxel is free, none is hit
    L = row(20.0, 0.0)
    assert np.array_equal(L[4, 4], np.full(8, lm, np.float32)) and np.count_nonzero(L) == 8
    # a depth before the start of the walk: nothing
    o2 = np.array([[-1.5], [0.5], [0.5]], np.float32)
    assert np.count_nonzero(row(-1.0, 0.0, oo=o2)) == 0
    # a ray along -z from inside: the same rule in the other direction
    o3 = np.array([[0.5], [0.5], [3.5]], np.float32)
    d3 = np.array([[0.0], [0.0], [-1.0]], np.float32)
    L = row(5.2, 0.0, oo=o3, dd=d3)          # z = -1.7: voxel 2
    assert np.array_equal(L[:, 4, 4], np.array([0, 0, lh] + [lm] * 5, np.float32))


def test_occupancy_one_measurement_per_voxel_per_pose(orc):
    desc = orc.occ_desc(8, -4.0, 1.0)
    lh, lm = np.float32(orc.logit(0.7)), np.float32(orc.logit(0.4))
    o = np.array([[-3.9, -3.9, -3.9], [0.5, 0.5, 0.5], [0.5, 0.5, 0.5]], np.float32)
    d = np.array([[1.0] * 3, [0.0] * 3, [0.0] * 3], np.float32)
    # ray 0 ends in voxel 4 sharply, ray 1 ends there with U = 1 voxel, ray 2
    # passes through voxel 4 freely and ends in voxel 6
    D = np.array([4.4, 4.4, 6.4], np.float32)
    U = np.array([0.0, 1.0, 0.0], np.float32)
    A = np.ones(3, np.float32)
    for perm in ([0, 1, 2], [2, 1, 0], [1, 2, 0]):
        L = np.zeros((8, 8, 8), np.float32)
        orc.occupancy_update(desc, L, o[:, perm], d[:, perm], D[perm], U[perm], A[perm])
        # voxel 4: the strongest hit, never the miss; voxel 5 free; voxel 6 hit
        assert np.array_equal(L[4, 4], np.array([lm] * 4 + [lh, lm, lh, 0], np.float32)), perm


def _all_segments(n, lo, vs, o, d):
    """Entry and exit distance of the ray through every voxel, FP64 slab test."""
    sc = type("G", (), {})()
    sc.n, sc.lo, sc.voxel = n, lo, vs
    sc.occupied = np.ones((n, n, n), bool)
    sc.field_map = np.zeros((n, n, n), np.int32)
    _, _, _, tin, tout = brute_segments(sc, o, d)
    return tin, tout


def test_occupancy_matches_brute_force(orc):
    n, lo, vs = 6, -1.5, 0.5
    desc = orc.occ_desc(n, lo, vs)
    lh, lm = orc.logit(0.7), orc.logit(0.4)
    rng = np.random.default_rng(11)
    checked = 0
    for r in range(300):
        o = rng.uniform(-1.4, 1.4, size=3).astype(np.float32)
        dv = rng.normal(size=3); dv /= np.linalg.norm(dv)
        dv = dv.astype(np.float32)
        D = np.float32(rng.uniform(0.2, 3.0)); U = np.float32(rng.uniform(0.0, 0.6))
        tin, tout = _all_segments(n, lo, vs, o, dv)
        tin = np.maximum(tin, 0.0)
        e = float(np.float32(D - U))
        pos = tout > tin
        margins = np.concatenate([np.abs(tout[pos] - e), np.abs(tin[pos] - D), np.abs(tout[pos] - D),
                                  (tout - tin)[pos]])
        if np.min(margins) < 1e-4:
            continue
        L = np.zeros((n, n, n), np.float32)
        orc.occupancy_update(desc, L, o[:, None], dv[:, None], np.array([D]), np.array([U]), np.array([1.0]))
        want = np.zeros((n, n, n))
        hit = pos & (tin <= D) & (D < tout)
        free = pos & (tout <= e)
        want[free] = lm
        want[hit] = lh / (1.0 + float(U) / vs)
        assert hit.sum() <= 1
        assert np.allclose(L, want, rtol=0, atol=1e-6), r
        checked += 1
    assert checked > 200


def test_occupancy_invariants_over_poses(orc):
    n = 16
    desc = orc.occ_desc(n, -4.0, 0.5)
    rng = np.random.default_rng(5)
    L = np.zeros((n, n, n), np.float32)
    walked = np.zeros((n, n, n), bool)
    for pose in range(8):
        N = 1500
        c = rng.uniform(-3, 3, size=3)
        o = np.repeat(c[:, None], N, axis=1).astype(np.float32)
        dv = rng.normal(size=(3, N)); dv /= np.linalg.norm(dv, axis=0)
        dv = dv.astype(np.float32)
        D = rng.uniform(0.5, 6.0, N).astype(np.float32)
        U = rng.uniform(0.0, 1.0, N).astype(np.float32)
        A = rng.uniform(0.0, 1.0, N).astype(np.float32)
        before = L.copy()
        p = orc.occupancy_update(desc, L, o, dv, D, U, A)
        assert L.min() >= -2.0 and L.max() <= 3.5
        walked |= L != before
        # probability is the logistic of the logit
        assert np.allclose(np.log(p / (1 - p)), L, rtol=0, atol=2e-6)
    # voxels no ray reached keep their initial value
    assert np.all(L[~walked] == 0)
    assert 0 < walked.sum() < n ** 3


def test_global_measure_opaque_first_sample(orc):
    lay = synth.global_mlp_layout(16, color_width=8)
    w = np.zeros(synth.n_params(lay), np.float32)
    t = synth.unpack(lay, w)
    o = np.zeros((3, 4), np.float32)
    d = np.array([[1, 0, 0, 0.6], [0, 1, 0, 0.8], [0, 0, 1, 0]], np.float32)
    # a huge constant density puts all the weight on the first sample (t = near)
    t["bs"][0] = 1e5
    D, U, A = orc.global_measure(w, o, d, n_samples=16, width=16, color_width=8)
    assert np.allclose(D, 0.1, atol=1e-7) and np.all(U < 1e-6) and np.allclose(A, 1.0)
    # zero density: no measurement
    t["bs"][0] = 0.0
    D, U, A = orc.global_measure(w, o, d, n_samples=16, width=16, color_width=8)
    assert np.all(A == 0) and np.all(D == 0) and np.all(U == 0)
    # a constant density c along the ray: against the compositing of the step
    t["bs"][0] = 0.3
    ts, dl = orc.invdepth_t(16, 0.1, 20.0)
    D, U, A = orc.global_measure(w, o, d, n_samples=16, width=16, color_width=8)
    tau = 0.3 * dl.astype(np.float64)
    S = np.concatenate([[0.0], np.cumsum(tau)[:-1]])
    wts = np.exp(-S) * (1 - np.exp(-tau))
    assert np.allclose(A, 1 - np.exp(-tau.sum()), rtol=1e-12)
    assert np.allclose(D, (wts * ts).sum() / wts.sum(), rtol=1e-12)


# ---------------------------------------------------------------------------
# Stage II adaptive field assignment (Sec. 4.2, Alg.1) and the uniform variant
# ---------------------------------------------------------------------------

def _brute_assign(occ, thr, n):
    """Alg.1 Stage II over index triples in plain Python (tiny grids only)."""
    nz, ny, nx = occ.shape
    free = [(z, y, x) for z in range(nz) for y in range(ny) for x in range(nx) if occ[z, y, x] > thr]
    S = len(free)
    out = np.full(occ.shape, -1, np.int32)
    for k in range(n):
        sk = S // n + (1 if k < S % n else 0)
        if sk == 0:
            continue
        a = min(free)                       # (z, y, x) order is the linear order
        free.sort(key=lambda v: (sum((p - q) ** 2 for p, q in zip(v, a)), v))
        for v in free[:sk]:
            out[v] = k
        free = free[sk:]
    return out


def test_assign_line_of_voxels(orc):
    occ = np.ones((1, 1, 10), np.float32)
    fmap, S = orc.assign_fields(occ, 0.5, 3)
    # sizes 4, 3, 3 (the first S mod n fields take the extra voxel); each
    # anchor is the leftmost free voxel, its nearest free voxels lie to its right
    assert S == 10 and fmap.ravel().tolist() == [0, 0, 0, 0, 1, 1, 1, 2, 2, 2]
    fmap, _ = orc.assign_fields(occ, 0.5, 12)
    assert fmap.ravel().tolist() == list(range(10))          # more fields than voxels: ten singletons


def test_assign_euclidean_nearest_and_clusters(orc):
    occ = np.zeros((1, 4, 4), np.float32)
    occ[0, 0, 0] = occ[0, 2, 2] = occ[0, 0, 3] = 1.0
    fmap, _ = orc.assign_fields(occ, 0.5, 2)
    # from the anchor (0,0,0): (2,2) is at squared distance 8, (0,3) at 9, so
    # (2,2) joins the anchor (by grid steps the order would be the other way)
    assert fmap[0, 0, 0] == 0 and fmap[0, 2, 2] == 0 and fmap[0, 0, 3] == 1
    occ = np.zeros((8, 8, 8), np.float32)
    occ[:2, :2, :2] = 1.0
    occ[6:, 6:, 6:] = 1.0
    fmap, S = orc.assign_fields(occ, 0.5, 2)
    assert S == 16 and np.all(fmap[:2, :2, :2] == 0) and np.all(fmap[6:, 6:, 6:] == 1)
    assert np.all(fmap[occ == 0] == -1)


def test_assign_matches_brute_force(orc):
    for seed, shape, p, n in ((1, (3, 4, 5), 0.5, 4), (2, (6, 6, 6), 0.3, 7), (3, (5, 2, 7), 0.8, 3),
                              (4, (4, 4, 4), 0.05, 9)):
        occ = np.random.default_rng(seed).uniform(size=shape).astype(np.float32)
        fmap, S = orc.assign_fields(occ, 1 - p, n)
        assert S == int((occ > 1 - p).sum())
        assert np.array_equal(fmap, _brute_assign(occ, 1 - p, n)), seed


def test_assign_sizes_and_nearest_property(orc):
    occ = np.random.default_rng(7).uniform(size=(10, 12, 9)).astype(np.float32)
    n = 13
    fmap, S = orc.assign_fields(occ, 0.6, n)
    sizes = np.bincount(fmap[fmap >= 0], minlength=n)
    assert sizes.sum() == S and set(sizes.tolist()) <= {S // n, S // n + 1}
    assert np.all(sizes[: S % n] == S // n + 1)
    z, y, x = np.nonzero(fmap >= 0)
    lin = x + 9 * (y + 12 * z)
    lab = fmap[z, y, x]
    for k in range(n):
        mine = lab == k
        later = lab > k
        a = lin[mine].min()
        assert not np.any(lin[later] < a)                 # the anchor is the smallest free index
        az, ay, ax = a // (9 * 12), (a // 9) % 12, a % 9
        d2 = (x - ax) ** 2 + (y - ay) ** 2 + (z - az) ** 2
        worst = max(zip(d2[mine], lin[mine]))
        assert all((dd, ll) > worst for dd, ll in zip(d2[later], lin[later]))   # nobody later was nearer


def test_assign_uniform_blocks(orc):
    occ = np.ones((4, 4, 4), np.float32)
    fmap, nf = orc.assign_uniform(occ, 0.5, (2, 2, 2))
    z, y, x = np.indices((4, 4, 4))
    assert nf == 8 and np.array_equal(fmap, x // 2 + 2 * (y // 2) + 4 * (z // 2))
    # only non-empty blocks become fields, numbered in block order
    occ = np.zeros((4, 4, 4), np.float32)
    occ[3, 0, 3] = 1.0          # block (1, 0, 1) = 5
    occ[0, 3, 1] = 1.0          # block (0, 1, 0) = 2
    fmap, nf = orc.assign_uniform(occ, 0.5, (2, 2, 2))
    assert nf == 2 and fmap[0, 3, 1] == 0 and fmap[3, 0, 3] == 1 and (fmap >= 0).sum() == 2
    # a side of 5 cut into 2 blocks: indices 0..2 and 3..4 (floor(i * 2 / 5))
    occ = np.ones((1, 1, 5), np.float32)
    fmap, nf = orc.assign_uniform(occ, 0.5, (2, 1, 1))
    assert nf == 2 and fmap.ravel().tolist() == [0, 0, 0, 1, 1]
    fmap, nf = orc.assign_uniform(np.ones((3, 3, 3), np.float32), 0.5, (1, 1, 1))
    assert nf == 1 and np.all(fmap == 0)


# ---------------------------------------------------------------------------
# Distillation of the global field into the local fields (Sec. 4.2, Eq.7)
# ---------------------------------------------------------------------------

def _distill_points(M, n_fields, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-3.5, 3.5, size=(3, M)).astype(np.float32)
    d = rng.normal(size=(3, M)); d /= np.linalg.norm(d, axis=0)
    field = rng.integers(0, n_fields, M).astype(np.int32)
    ts = rng.uniform(0, 3, M).astype(np.float32)
    tr = rng.uniform(0, 1, (3, M)).astype(np.float32)
    return x, d.astype(np.float32), field, ts, tr


def test_distill_constant_fields_closed_form(orc):
    """Zero weights leave sigma = softplus(b_s) and c = sigmoid(b_4) per field,
    so Eq.7 and its bias gradients are closed forms; each field's term is
    averaged over its own points."""
    sc = synth.tiny_scene(4, 3, p_occ=0.5, n_fields=2, hidden=8)
    lay = synth.local_mlp_layout(8)
    w = np.zeros((2, synth.n_params(lay)), np.float32)
    bs = [0.3, -1.2]
    b4 = [[0.1, -0.4, 0.7], [-0.2, 0.5, 0.0]]
    for k in range(2):
        t = synth.unpack(lay, w[k])
        t["bs"][0] = bs[k]; t["b4"][:] = b4[k]
    x, d, field, ts, tr = _distill_points(11, 2, 4)
    field[:3] = 0; field[3:] = 1                       # I_0 = 3, I_1 = 8
    loss, grad, sig, rgb = orc.distill(sc, x, d, field, ts, tr, weights=w)
    ts, tr = ts.astype(np.float64), tr.astype(np.float64)
    want, g_bs, g_b4 = 0.0, [0.0, 0.0], [[0.0] * 3, [0.0] * 3]
    for k, I in ((0, 3), (1, 8)):
        s = sp(float(np.float32(bs[k])))
        c = [1 / (1 + math.exp(-float(np.float32(v)))) for v in b4[k]]
        for i in np.nonzero(field == k)[0]:
            want += ((s - ts[i]) ** 2 + sum((c[q] - tr[q, i]) ** 2 for q in range(3))) / I
            g_bs[k] += 2 * (s - ts[i]) / I / (1 + math.exp(-float(np.float32(bs[k]))))
            for q in range(3):
                g_b4[k][q] += 2 * (c[q] - tr[q, i]) / I * c[q] * (1 - c[q])
    assert abs(loss - want) < 1e-12 * max(1, want)
    for k in range(2):
        gk = synth.unpack(lay, grad[k].copy())
        assert abs(gk["bs"][0] - g_bs[k]) < 1e-12
        assert np.allclose(gk["b4"], g_b4[k], rtol=0, atol=1e-12)
        assert np.all(gk["W1"] == 0) and np.all(gk["W3"] == 0)    # zero weights pass no gradient further back
    assert np.allclose(sig[:3], sp(float(np.float32(bs[0])))) and np.allclose(sig[3:], sp(float(np.float32(bs[1]))))


def test_distill_finite_difference_and_ignored_points(orc):
    sc = synth.tiny_scene(4, 6, p_occ=0.5, n_fields=3, hidden=16)
    rng = np.random.default_rng(6)
    w0 = sc.weights + rng.normal(size=sc.weights.shape).astype(np.float32) * 0.05
    x, d, field, ts, tr = _distill_points(40, 3, 7)
    loss, grad, _, _ = orc.distill(sc, x, d, field, ts, tr, weights=w0)
    flat = w0.ravel()

    def loss_fn(wf):
        return orc.distill(sc, x, d, field, ts, tr, weights=wf.reshape(w0.shape))[0]
    idx = rng.choice(flat.size, 120, replace=False)
    bad = _fd_check(loss_fn, flat, idx, grad.ravel())
    assert not bad, bad[:5]
    # points whose field id is out of range take no part
    f2 = np.concatenate([field, np.array([-1, 3], np.int32)])
    x2 = np.concatenate([x, x[:, :2]], axis=1); d2 = np.concatenate([d, d[:, :2]], axis=1)
    l2, g2, _, _ = orc.distill(sc, x2, d2, f2, np.concatenate([ts, ts[:2]]), np.concatenate([tr, tr[:, :2]], axis=1),
                               weights=w0)
    assert abs(l2 - loss) <= 1e-13 * loss and np.allclose(g2, grad, rtol=1e-12, atol=1e-15)


def test_global_points_constant_field(orc):
    lay = synth.global_mlp_layout(16, color_width=8)
    w = np.zeros(synth.n_params(lay), np.float32)
    t = synth.unpack(lay, w)
    t["bs"][0] = 0.75; t["b11"][:] = [0.2, -0.1, 0.4]
    x, d, _, _, _ = _distill_points(5, 1, 8)
    sig, rgb = orc.global_points(w, x, d, width=16, color_width=8)
    assert np.all(sig == np.float64(np.float32(0.75)))
    assert np.allclose(rgb.T, [sg(float(np.float32(v))) for v in (0.2, -0.1, 0.4)], atol=1e-15)
    # the raw position reaches the density through the first layer's identity slot
    t["W1"][0, 2] = 1.0; t["W2"][0, 0] = 1.0; t["W3"][0, 0] = 1.0; t["W4"][0, 0] = 1.0
    t["W5"][0, 0] = 1.0; t["W6"][0, 0] = 1.0; t["W7"][0, 0] = 1.0; t["W8"][0, 0] = 1.0; t["ws"][0, 0] = 1.0
    sig, _ = orc.global_points(w, x, d, width=16, color_width=8)
    z = x[2].astype(np.float64) / 4.0
    assert np.allclose(sig, 0.75 + np.maximum(z, 0.0), atol=1e-7)


# ---------------------------------------------------------------------------
# Several samples per occupied voxel (a renderer variant of Sec. 4.2's dense
# sampling of the occupied voxels)
# ---------------------------------------------------------------------------

def test_samples_per_voxel_axis_ray(orc):
    sc = synth.tiny_scene(8, 5, p_occ=1.0, max_samples=64)
    sc.samples_per_voxel = 4
    o = np.array([[-3.9], [0.1], [0.2]], np.float32)
    d = np.array([[1.0], [0.0], [0.0]], np.float32)
    smp = orc.sample_rays(sc, o, d)
    assert smp["counts"][0] == 32
    # full voxels [t, t + 1) of unit length: quarter pieces, midpoints at
    # t + 1/8, 3/8, 5/8, 7/8 exactly
    t_mid, dl = smp["t_mid"][4:].reshape(7, 4), smp["delta"][4:].reshape(7, 4)
    t_in = np.float32(0.9) + np.arange(7, dtype=np.float32)
    assert np.all(dl == np.float32(0.25))
    for q, frac in enumerate((0.125, 0.375, 0.625, 0.875)):
        assert np.allclose(t_mid[:, q], t_in + frac, rtol=0, atol=2e-7)
    assert list(smp["voxel"][::4]) == [i + 8 * (4 + 8 * 4) for i in range(8)]
    # one sample per voxel is the midpoint rule, unchanged
    sc.samples_per_voxel = 1
    one = orc.sample_rays(sc, o, d)
    assert np.array_equal(one["t_mid"], orc.sample_rays(synth.tiny_scene(8, 5, p_occ=1.0, max_samples=64), o, d)["t_mid"])


def test_samples_per_voxel_lengths_and_cap(orc):
    sc = synth.tiny_scene(8, 7, p_occ=0.5, max_samples=256)
    rng = np.random.default_rng(7)
    N = 200
    o = rng.uniform(-3.5, 3.5, size=(3, N)).astype(np.float32)
    d = rng.normal(size=(3, N)); d /= np.linalg.norm(d, axis=0); d = d.astype(np.float32)
    base = orc.sample_rays(sc, o, d)
    sc.samples_per_voxel = 3
    three = orc.sample_rays(sc, o, d)
    assert np.array_equal(three["counts"], 3 * base["counts"])
    # the pieces of each voxel tile its segment: lengths add up, midpoints
    # increase inside it
    dl = three["delta"].reshape(-1, 3).astype(np.float64)
    assert np.allclose(dl.sum(axis=1), base["delta"], rtol=1e-6, atol=1e-7)
    tm = three["t_mid"].reshape(-1, 3)
    assert np.all(np.diff(tm, axis=1) > 0)
    lo = base["t_mid"] - 0.5 * base["delta"]; hi = base["t_mid"] + 0.5 * base["delta"]
    assert np.all((tm >= lo[:, None] - 1e-6) & (tm <= hi[:, None] + 1e-6))
    # the cap counts pieces: a voxel may be cut off part-way
    sc.max_samples = 5
    capped = orc.sample_rays(sc, o, d)
    assert np.array_equal(capped["counts"], np.minimum(three["counts"], 5))


# ---------------------------------------------------------------------------
# Omni-directional stereo rays (stereoscopic mode, Sec. 5)
# ---------------------------------------------------------------------------

def test_ods_rays_geometry(orc):
    W, H, eye = 65, 32, np.float32(0.032)
    mono_o, mono_d = orc.equirect_rays(W, H, synth.IDENTITY_C2W)
    o0, d0 = orc.ods_rays(W, H, synth.IDENTITY_C2W, 0.0)
    assert np.array_equal(o0, mono_o) and np.array_equal(d0, mono_d)
    oR, dR = orc.ods_rays(W, H, synth.IDENTITY_C2W, eye)
    oL, dL = orc.ods_rays(W, H, synth.IDENTITY_C2W, -eye)
    assert np.array_equal(dR, mono_d) and np.array_equal(dL, mono_d)
    assert np.array_equal(oL, -oR)                              # the two eyes mirror through the centre
    off = oR.astype(np.float64)
    assert np.allclose(np.linalg.norm(off, axis=0), eye, rtol=1e-6)
    assert np.all(off[1] == 0)                                  # on the horizontal viewing circle
    # perpendicular to the ray's horizontal heading
    assert np.abs(off[0] * mono_d[0] + off[2] * mono_d[2]).max() < 1e-7
    # looking along +z (the centre column of an odd width) the right eye sits at +x
    mid = (H // 2) * W + W // 2
    assert abs(mono_d[0, mid]) < 1e-7 and mono_d[2, mid] > 0.99
    assert abs(off[0, mid] - eye) < 1e-9 and abs(off[2, mid]) < 1e-9
    # a camera moved and turned a quarter: the offsets turn with it
    c2w = synth.c2w_yaw((1.0, 2.0, 3.0), 1)
    o1, _ = orc.ods_rays(W, H, c2w, eye)
    R = c2w.reshape(3, 4)[:, :3].astype(np.float64)
    assert np.allclose(o1.astype(np.float64) - np.array([[1.0], [2.0], [3.0]]), R @ off, atol=1e-6)


# ---------------------------------------------------------------------------
# Per-field encoding frames (a renderer variant: each field encodes its box)
# ---------------------------------------------------------------------------

def test_field_frames_boxes(orc):
    fm = np.full((8, 8, 8), -1, np.int32)
    fm[0:4, 1, 2:6] = 0                      # z 0..3, y 1, x 2..5
    fm[7, 7, 7] = 2                          # a single voxel; field 1 is empty
    fr = orc.field_frames(fm, -4.0, 1.0, 3)
    assert np.array_equal(fr[0], np.float32([0.0, -2.5, -2.0, 2.0]))
    assert np.array_equal(fr[1], np.float32([0.0, 0.0, 0.0, 1.0]))
    assert np.array_equal(fr[2], np.float32([3.5, 3.5, 3.5, 0.5]))
    # random maps against the index extremes found by numpy
    rng = np.random.default_rng(3)
    fm = rng.integers(-1, 5, size=(6, 7, 9)).astype(np.int32)
    fr = orc.field_frames(fm, (-1.0, -2.0, -0.5), 0.25, 5)
    for f in range(5):
        z, y, x = np.nonzero(fm == f)
        lo = np.array([-1.0, -2.0, -0.5]) + 0.25 * np.array([x.min(), y.min(), z.min()])
        hi = np.array([-1.0, -2.0, -0.5]) + 0.25 * (np.array([x.max(), y.max(), z.max()]) + 1)
        assert np.allclose(fr[f, :3], (lo + hi) / 2, atol=1e-7) and abs(fr[f, 3] - ((hi - lo) / 2).max()) < 1e-7


def test_field_frames_reach_the_encoding(orc):
    """A field wired to output softplus(relu(xhat_x)) shows which frame
    encodes its points."""
    sc = synth.tiny_scene(4, 9, p_occ=1.0, n_fields=2, hidden=8)
    lay = synth.local_mlp_layout(8)
    w = np.zeros((2, synth.n_params(lay)), np.float32)
    for k in range(2):
        t = synth.unpack(lay, w[k])
        t["W1"][0, 0] = 1.0; t["W2"][0, 0] = 1.0; t["ws"][0, 0] = 1.0
    x = np.array([[1.5, 3.0, -2.0], [0.25, 0.5, 0.75], [0.0, 1.0, 2.0]], np.float32)
    d = np.tile(np.float32([[0.0], [0.0], [1.0]]), (1, 3))
    field = np.array([0, 1, 1], np.int32)
    ts = np.zeros(3, np.float32); tr = np.zeros((3, 3), np.float32)
    _, _, sig, _ = orc.distill(sc, x, d, field, ts, tr, weights=w)
    want = [sp(max(0.0, float(v) / 4.0)) for v in x[0]]        # the scene frame: centre 0, half extent 4
    assert np.allclose(sig, want, atol=1e-12)
    sc.frames = np.array([[1.0, 0.0, 0.0, 0.25], [2.0, 0.0, 0.0, 2.0]], np.float32)
    _, _, sig, _ = orc.distill(sc, x, d, field, ts, tr, weights=w)
    want = [sp(max(0.0, (1.5 - 1.0) * 4.0)), sp(max(0.0, (3.0 - 2.0) * 0.5)), sp(0.0)]
    assert np.allclose(sig, want, atol=1e-12)
    # frames equal to the scene's reproduce the scene-wide encoding exactly
    sc.frames = np.array([[0.0, 0.0, 0.0, 4.0]] * 2, np.float32)
    w2 = sc.weights
    o, dd = orc.equirect_rays(32, 16, synth.IDENTITY_C2W)
    a = orc.render_rays(sc, o, dd)
    sc.frames = None
    b = orc.render_rays(sc, o, dd)
    assert all(np.array_equal(p, q) for p, q in zip(a, b)) and w2 is sc.weights


# ---------------------------------------------------------------------------
# Early ray termination (a stopping rule of Eq.5's compositing)
# ---------------------------------------------------------------------------

def test_termination_drops_less_than_the_transmittance(orc):
    """Compositing telescopes: the weights after the first K samples sum to
    T_K - T_final <= T_K = 1 - (opacity of the first K samples), and colours
    lie in [0, 1], so the K-sample render differs from the full one by at
    most T_K in every channel, in opacity by T_K - T_final exactly."""
    sc = synth.scene_small()
    o, d = orc.equirect_rays(64, 32, synth.IDENTITY_C2W)
    K = 3
    full = orc.render_rays(sc, o, d)
    first = orc.render_rays(sc, o, d, max_samples=K)
    T_K = 1.0 - first[2]
    assert (np.abs(full[0] - first[0]) <= T_K[None, :] + 1e-12).all()
    assert (full[2] - first[2] <= T_K + 1e-12).all() and (full[2] >= first[2] - 1e-12).all()
    assert (T_K < 0.999).any() and (np.abs(full[0] - first[0]).max() > 1e-6)   # the test is not vacuous


def test_termination_rule_selects_per_ray(orc):
    sc = synth.scene_small()
    o, d = orc.equirect_rays(64, 32, synth.IDENTITY_C2W)
    K = 3
    full = orc.render_rays(sc, o, d)
    first = orc.render_rays(sc, o, d, max_samples=K)
    counts = np.diff(orc.sample_rays(sc, o, d)["offsets"])
    T_K = 1.0 - first[2]
    eps = float(np.median(T_K[counts > K]))          # about half of the long rays stop
    rgb, depth, opac, stopped = orc.render_rays_terminated(sc, o, d, eps, K)
    assert stopped.any() and (~stopped & (counts > K)).any()
    assert np.array_equal(stopped, (counts > K) & (T_K < eps))
    assert np.array_equal(rgb[:, stopped], first[0][:, stopped]) and np.array_equal(rgb[:, ~stopped], full[0][:, ~stopped])
    assert np.array_equal(opac[stopped], first[2][stopped]) and np.array_equal(depth[~stopped], full[1][~stopped])
    # eps = 0 keeps every sample
    rgb0, _, _, st0 = orc.render_rays_terminated(sc, o, d, 0.0, K)
    assert not st0.any() and np.array_equal(rgb0, full[0])
