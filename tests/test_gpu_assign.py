"""GPU Stage II field assignment (Sec. 4.2, Alg.1) and the uniform block
decomposition against the oracle: integer work, compared bit for bit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_02705_amd import assign
    return assign


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("shape,p,n", [((1, 1, 10), 1.0, 3), ((3, 4, 5), 0.5, 4), ((6, 6, 6), 0.3, 7),
                                       ((5, 2, 7), 0.8, 30), ((7, 9, 11), 0.4, 1), ((4, 4, 4), 0.05, 9),
                                       ((8, 8, 8), 0.0, 5), ((33, 17, 29), 0.35, 57), ((1, 1, 1), 1.0, 1),
                                       ((1, 1, 2), 1.0, 2), ((1, 1, 600), 0.6, 7), ((2, 3, 520), 0.5, 13),
                                       ((1, 1, 2100), 0.5, 9), ((1100, 2, 1), 0.7, 6)])
def test_assign_small_grids_match_oracle(A, orc, shape, p, n):
    u = synth.uniform(len(shape) + n, synth.STREAM_SCENE, np.arange(int(np.prod(shape)), dtype=np.uint64))
    occ = u.astype(np.float32).reshape(shape)
    thr = float(np.float32(1 - p)) if p < 1.0 else -1.0
    fmap, S = A.assign_fields(_t(occ), thr, n)
    ref, rS = orc.assign_fields(occ, thr, n)
    assert S == rS
    assert np.array_equal(_np(fmap), ref)


def test_assign_room_scene_matches_oracle(A, orc):
    """The headline scene's 128^3 occupancy (137,929 occupied voxels) into
    141 fields, as many as its octree split gives."""
    sc = synth.scene_room(with_weights=False)
    occ = sc.occ.astype(np.float32)
    fmap, S = A.assign_fields(_t(occ), sc.threshold, 141)
    ref, rS = orc.assign_fields(occ, sc.threshold, 141)
    assert S == rS == int(sc.occupied.sum())
    got = _np(fmap)
    assert np.array_equal(got, ref)
    sizes = np.bincount(got[got >= 0], minlength=141)
    assert set(sizes.tolist()) <= {S // 141, S // 141 + 1}


def test_assign_deterministic(A, orc):
    occ = synth.uniform(9, synth.STREAM_SCENE, np.arange(40 ** 3, dtype=np.uint64)).astype(np.float32)
    occ = occ.reshape(40, 40, 40)
    a, _ = A.assign_fields(_t(occ), 0.8, 64)
    b, _ = A.assign_fields(_t(occ), 0.8, 64)
    assert np.array_equal(_np(a), _np(b))


@pytest.mark.parametrize("shape,blocks", [((4, 4, 4), (2, 2, 2)), ((1, 1, 5), (2, 1, 1)), ((13, 7, 29), (3, 7, 5)),
                                          ((128, 128, 128), (6, 6, 6)), ((16, 16, 16), (1, 1, 1))])
def test_assign_uniform_matches_oracle(A, orc, shape, blocks):
    u = synth.uniform(3, synth.STREAM_SCENE, np.arange(int(np.prod(shape)), dtype=np.uint64))
    occ = u.astype(np.float32).reshape(shape)
    fmap, nf = A.assign_uniform(_t(occ), 0.9, blocks)
    ref, rnf = orc.assign_uniform(occ, 0.9, blocks)
    assert nf == rnf
    assert np.array_equal(_np(fmap), ref)


def test_assigned_map_renders(A, orc):
    """The adaptive map drives the renderer: a scene built on it samples and
    labels exactly as the oracle's scene with the oracle's map."""
    from paper_2208_02705_amd import render
    sc = synth.scene_small()
    occ = sc.occ.astype(np.float32)
    fmap, S = A.assign_fields(_t(occ), sc.threshold, sc.n_fields)
    ref, _ = orc.assign_fields(occ, sc.threshold, sc.n_fields)
    assert np.array_equal(_np(fmap), ref)
    scene = render.Scene(_t(occ), fmap, _t(sc.weights), lo=(sc.lo,) * 3, voxel=sc.voxel, threshold=sc.threshold,
                         hidden=sc.hidden, center=sc.center, half_extent=sc.half_extent)
    scene.near, scene.far, scene.max_samples = sc.near, sc.far, sc.max_samples
    o, d = orc.equirect_rays(64, 32, synth.IDENTITY_C2W)
    smp = render.sample_rays(scene, _t(o), _t(d))
    sc.field_map = ref
    want = orc.sample_rays(sc, o, d)
    assert np.array_equal(_np(smp["field"]), want["field"])
    scene.close()


def test_assign_large_scene_matches_oracle(A, orc):
    """The large configuration's 256^3 occupancy (1,142,256 occupied voxels)
    into 512 fields."""
    sl = synth.scene_large()
    occ = sl.occ.astype(np.float32)
    fmap, S = A.assign_fields(_t(occ), sl.threshold, 512)
    ref, rS = orc.assign_fields(occ, sl.threshold, 512)
    assert S == rS
    assert np.array_equal(_np(fmap), ref)
