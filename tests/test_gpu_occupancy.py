"""GPU Stage I occupancy (Sec. 4.1, Eq.6, Alg.1) against the oracle.

The update is specified in FP32 (the sampler's voxel walk, the band edge
D - U, the hit logit l_hit / (1 + U / voxel), the clamped logit sum), so the
logit grid must match the oracle bit for bit; the probability 1 / (1 + e^-l)
is FP32 on the GPU against the correctly rounded value (4 ulp). The depth
statistics are FP32 sums against FP64: 2e-6 in opacity and 2e-5 of the
sample range in depth and spread (a few roundings per term over at most a
few hundred terms). The global-field measurement inherits the BF16
tolerances of the global stage: opacity within 2e-2; the normalised
weights then carry a relative error up to about 2 * 2e-2 / A (weights and
their sum), which moves depth and spread by at most that times the spread
U about the depth, plus the 3e-2 floor of the global forward."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_02705_amd import occupancy
    return occupancy


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _samples(N, S, seed):
    """Increasing sample distances with their spacings and densities: every
    ninth ray empty, every seventh with one nearly opaque sample."""
    u = synth.uniform(seed, synth.STREAM_NOISE, np.arange(2 * N * S, dtype=np.uint64)).reshape(2, N, S)
    t = (0.1 + np.cumsum(0.02 + 0.2 * u[0], axis=1)).astype(np.float32)
    delta = np.diff(t, axis=1, append=t[:, -1:] + 0.05).astype(np.float32)
    sigma = (3.0 * u[1] ** 4).astype(np.float32)
    sigma[::9] = 0.0
    sigma[3::7, S // 2] = 1e4
    return t, delta, sigma


@pytest.mark.parametrize("S", [1, 2, 37, 64, 128, 200])
def test_depth_uncertainty_matches_oracle(M, orc, S):
    N = 1001                                  # a ragged last block (4 rays per block)
    t, delta, sigma = _samples(N, S, 40 + S)
    D, U, A = (_np(x) for x in M.depth_uncertainty(_t(t), _t(delta), _t(sigma)))
    rD, rU, rA = orc.depth_stats(t, delta, sigma)
    scale = float(t.max())
    assert np.abs(A - rA).max() <= 2e-6
    assert np.abs(D - rD).max() <= 2e-5 * scale
    assert np.abs(U - rU).max() <= 2e-5 * scale
    empty = ~sigma.any(axis=1)
    assert empty.sum() > 50 and np.all(A[empty] == 0) and np.all(D[empty] == 0) and np.all(U[empty] == 0)


def _grid_rays(orc, N, seed, centre):
    o = np.repeat(np.asarray(centre, np.float32)[:, None], N, axis=1)
    return o, synth.random_unit_dirs(N, seed)


def _compare(orc, M, om, desc, o, d, D, U, A, L_ref):
    om.update(_t(o), _t(d), _t(D), _t(U), _t(A))
    p_ref = orc.occupancy_update(desc, L_ref, o, d, D, U, A)
    L = _np(om.logit)
    assert np.array_equal(L.view(np.uint32), L_ref.view(np.uint32)), int((L != L_ref).sum())
    p = _np(om.prob)
    assert np.abs(p - p_ref).max() <= 4 * np.finfo(np.float32).eps
    return L


def test_occupancy_update_matches_oracle_over_poses(M, orc):
    n, lo, vs = 32, -4.0, 0.25
    om = M.OccupancyMap(n, lo, vs)
    desc = orc.occ_desc(n, lo, vs)
    L_ref = np.zeros((n, n, n), np.float32)
    # a voxel corner, inside, outside the box, then three more inside
    centres = [(0.0, 0.0, 0.0), (1.3, -0.7, 2.1), (-6.0, 0.3, 0.2), (0.1, 0.2, 0.3), (-0.4, 0.1, 0.0),
               (0.2, -0.3, -0.1)]
    for k, c in enumerate(centres):
        N = 20000
        o, d = _grid_rays(orc, N, 100 + k, c)
        D, U, A = synth.occupancy_measurements(N, 200 + k, d_hi=12.0, u_max=0.6)
        # awkward measurements and rays
        D[:10] = np.inf; U[10:20] = -0.1; U[20:30] = np.nan; o[:, 30:40] = np.nan
        D[40:50] = 0.0; U[40:50] = 0.0
        d[:, 50:60] = np.array([[1.0], [0.0], [0.0]], np.float32)       # axis-aligned
        d[:, 60:70] = np.array([[0.0], [-1.0], [0.0]], np.float32)
        L = _compare(orc, M, om, desc, o, d, D, U, A, L_ref)
    # free space seen from six positions saturates at the lower bound
    assert L.min() == np.float32(-2.0) and L.max() <= np.float32(3.5)


def test_occupancy_update_non_cubic_grid_and_far_clip(M, orc):
    n, lo, vs = (40, 24, 16), (-2.5, -1.5, -1.0), 0.125
    om = M.OccupancyMap(n, lo, vs, near=0.05, far=2.0, p_hit=0.8, p_miss=0.3, min_opacity=0.25)
    desc = orc.occ_desc(n, lo, vs, near=0.05, far=2.0, p_hit=0.8, p_miss=0.3, min_opacity=0.25)
    L_ref = np.zeros((16, 24, 40), np.float32)
    for k in range(2):
        N = 7777
        o, d = _grid_rays(orc, N, 300 + k, (0.1 * k, 0.2, -0.3))
        D, U, A = synth.occupancy_measurements(N, 400 + k, d_hi=3.0, u_max=0.3)
        _compare(orc, M, om, desc, o, d, D, U, A, L_ref)
    # a single ray
    o, d = _grid_rays(orc, 1, 9, (0.0, 0.0, 0.0))
    _compare(orc, M, om, desc, o, d, np.array([1.0], np.float32), np.array([0.0], np.float32),
             np.array([1.0], np.float32), L_ref)


def test_occupancy_update_is_order_independent(M, orc):
    import torch
    n, lo, vs = 32, -4.0, 0.25
    N = 30000
    o, d = _grid_rays(orc, N, 7, (0.4, 0.1, -0.2))
    D, U, A = synth.occupancy_measurements(N, 8, d_hi=6.0)
    perm = np.random.default_rng(0).permutation(N)
    a = M.OccupancyMap(n, lo, vs); b = M.OccupancyMap(n, lo, vs)
    a.update(_t(o), _t(d), _t(D), _t(U), _t(A))
    b.update(_t(o[:, perm]), _t(d[:, perm]), _t(D[perm]), _t(U[perm]), _t(A[perm]))
    assert torch.equal(a.logit, b.logit) and torch.equal(a.prob, b.prob)


def test_occupancy_full_panorama_matches_oracle(M, orc):
    """One sampling position at the headline size: a 2048 x 1024 equirect
    from the room scene's first camera centre into the 128^3 grid."""
    sc = synth.scene_room(with_weights=False)
    c = synth.camera_centres(sc, 1)[0]
    o, d = orc.equirect_rays(2048, 1024, synth.c2w_at(c))
    N = o.shape[1]
    D, U, A = synth.occupancy_measurements(N, 11, d_lo=0.3, d_hi=6.0, u_max=0.3, p_valid=0.95)
    om = M.OccupancyMap(128, -4.0, 0.0625)
    desc = orc.occ_desc(128, -4.0, 0.0625)
    L_ref = np.zeros((128, 128, 128), np.float32)
    _compare(orc, M, om, desc, o, d, D, U, A, L_ref)
    # a second position on top of the first
    c2 = synth.camera_centres(sc, 2)[1]
    o2, d2 = orc.equirect_rays(2048, 1024, synth.c2w_at(c2))
    D, U, A = synth.occupancy_measurements(N, 12, d_lo=0.3, d_hi=6.0, u_max=0.3, p_valid=0.95)
    _compare(orc, M, om, desc, o2, d2, D, U, A, L_ref)


def _global_batch(orc, N, seed):
    sc = synth.scene_room(with_weights=False)
    c = synth.camera_centres(sc, 1, seed=seed)[0]
    pix = (np.arange(N, dtype=np.int64) * 7919) % (2048 * 1024)
    return orc.equirect_rays(2048, 1024, synth.c2w_at(c), pix)


def test_global_measure_matches_oracle(M, orc):
    from paper_2208_02705_amd import render
    N = 64
    o, d = _global_batch(orc, N, 21)
    lay = synth.global_mlp_layout()
    w = synth.xavier_weights(lay, 1, 21, synth.STREAM_WEIGHTS)[0].astype(np.float32)
    gf = render.GlobalField()
    D, U, A = (_np(x) for x in M.global_measure(gf, _t(w), _t(o), _t(d), chunk=48))   # two chunks
    rD, rU, rA = orc.global_measure(w, o, d)
    print(f"measure: depth err {np.abs(D - rD).max():.3g}, spread err {np.abs(U - rU).max():.3g}, "
          f"opacity err {np.abs(A - rA).max():.3g}")
    assert np.abs(A - rA).max() <= 2e-2
    bound = 2 * 2e-2 / rA * rU + 3e-2
    assert np.all(np.abs(D - rD) <= bound), np.max(np.abs(D - rD) / bound)
    assert np.all(np.abs(U - rU) <= bound), np.max(np.abs(U - rU) / bound)
