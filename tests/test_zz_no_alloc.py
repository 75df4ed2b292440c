"""The allocation-free render entry point (r360_render_rays_noalloc: the
library's own device scratch array in place of a caller workspace) against
the workspace entry point r360_render_rays, through the C ABI. Both run the
same kernels over the same samples, so the outputs must agree bit for bit;
two calls in a row (the second with fewer rays, a ragged count) check that
what the first call left in the shared array does not leak into the second."""
import numpy as np
import pytest

import synth
from paper_2208_02705_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_02705_amd import render
    return render


def _rays(N, seed):
    rng = np.random.default_rng(seed)
    o = rng.uniform(-3, 3, size=(3, N)).astype(np.float32)
    d = rng.normal(size=(3, N)); d /= np.linalg.norm(d, axis=0)
    return o, d.astype(np.float32)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_render_equals_workspace_render(R, prec):
    import torch
    sc = synth.scene_room()
    scene = R.Scene.from_synth(sc)
    for N, seed in ((20000, 1), (3001, 2)):
        o, d = (torch.from_numpy(a).cuda() for a in _rays(N, seed))
        ref = R.render_rays(scene, o, d, precision=prec)
        out = tuple(torch.full_like(t, float("nan")) for t in ref)
        R.render_rays_noalloc(scene, o, d, *out, precision=prec)
        torch.cuda.synchronize()
        for a, b, name in zip(ref, out, ("rgb", "depth", "opacity")):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (prec, N, name)
        assert float(ref[2].max()) > 0.0      # some rays hit occupied voxels
    scene.close()


def test_noalloc_render_rejects_what_does_not_fit(R):
    import torch
    sc = synth.scene_room()
    scene = R.Scene.from_synth(sc)
    N = 200000                                   # 200,000 x 64 slots x 36 B > 128 MiB
    o, d = (torch.from_numpy(a).cuda() for a in _rays(N, 3))
    out = (torch.empty(3, N, device="cuda"), torch.empty(N, device="cuda"), torch.empty(N, device="cuda"))
    with pytest.raises(_lib.R360Error) as e:
        R.render_rays_noalloc(scene, o, d, *out)
    assert e.value.status == _lib.R360_EWORKSPACE
    opts = R._opts(scene, None, None, None, "fp32")
    opts.term_eps, opts.term_after = 0.01, 8
    import ctypes as C
    st = _lib.lib().r360_render_rays_noalloc(scene._h, R._ptr(o), R._ptr(d), N, C.byref(opts), R._ptr(out[0]),
                                             R._ptr(out[1]), R._ptr(out[2]), R._stream())
    assert st == _lib.R360_EUNSUPPORTED
    scene.close()
