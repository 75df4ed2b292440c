"""Gradients of the training step (Sec. 4.2: L2 photometric loss over the
rendered colours) on the room scene at hidden width 64, on the first 16 rays
of the 65,536-ray training batch (20 camera centres, teacher targets plus
N(0, 0.01^2) noise):

- central finite differences of the FP64 GPU forward over a seeded set of
  512 weights spread over every tensor of the fields those rays touch,
  against the FP64 GPU analytic gradient;
- the FP64 GPU analytic gradient against the oracle's, on every weight;
- the FP32 training-step gradient against the oracle's, per field and per
  tensor, and entry by entry.

Tolerance basis. Finite differences: with step h, the central difference of
an FP64 loss L carries a rounding error of at most about n u L / h (u = 2^-53,
n the roundings of one loss evaluation, a few hundred: NOISE counts 1,000)
and a truncation error of order h^2 L'''. At h = 3e-5 max(|w|, 0.1) the
rounding part stays near 1e-11 and the truncation part near 1e-9 of the
entry; a weight whose two estimates at h and h/2 disagree beyond that has a
ReLU kink inside the step (a sample's pre-activation crosses zero) and is
set aside, at most 10 % of them.
FP64 analytic gradients: both sides sum the same terms in FP64 in different
orders, so they agree to a few hundred ulps of the block's scale.
FP32 per entry: within 2e-4 of the oracle's magnitude plus its kink
magnitude at 1e-6 (the bound of test_gpu_backward.py).
BF16 is compared on the headline batch (test_gpu_backward.py), not here:
with teacher targets the residuals C - C* are about 2e-2 (the loss is their
mean square, 5e-4), the order of the BF16 colour error itself, so each
ray's dL/dC in BF16 carries an error of the order of its own size and the
gradient is not resolved below the largest entry's order.
"""
import numpy as np
import pytest

import synth
from tests._grad import block_errors, describe, magnitude_errors, training_rays, training_targets

pytestmark = pytest.mark.gpu

N_RAYS = 16
N_FD = 512
NOISE = 1000 * 2.0 ** -53


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_02705_amd import render
    return render


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def subset(orc):
    sc = synth.scene_room()
    o, d = training_rays(orc, sc, N_RAYS)
    tgt = training_targets(orc, sc, o, d)
    smp = orc.sample_rays(sc, o, d)
    fields = np.unique(smp["field"])
    return sc, o, d, tgt, fields


def test_training_subset_finite_differences(R, orc, subset):
    import torch
    sc, o, d, tgt, fields = subset
    assert len(fields) >= 4, fields
    scene = R.Scene.from_synth(sc)
    to, td, tt = _t(o), _t(d), torch.from_numpy(tgt.astype(np.float64)).cuda()
    w64 = torch.from_numpy(sc.weights.astype(np.float64)).cuda()
    P = sc.weights.shape[1]

    def loss_of(w):
        rgb = R.GradcheckFunction.apply(w, scene, to, td)
        return ((rgb - tt) ** 2).mean()

    wg = w64.clone().requires_grad_(True)
    loss_of(wg).backward()
    g_gpu = _np(wg.grad)

    # 512 weights: for each tensor of the layout, entries of the touched fields
    lay = synth.local_mlp_layout(sc.hidden)
    rng = np.random.default_rng(2208)
    per = -(-N_FD // len(lay))
    picks = []
    off = 0
    for name, shape in lay:
        size = int(np.prod(shape))
        fsel = rng.choice(fields, per)
        esel = rng.integers(0, size, per)
        picks += [(int(f), off + int(e), name) for f, e in zip(fsel, esel)]
        off += size
    assert off == P
    picks = picks[:N_FD]

    flat = w64.view(-1)
    top = float(np.abs(g_gpu).max())
    with torch.no_grad():
        L0 = float(loss_of(w64))
    rejected, bad, worst = 0, [], 0.0
    with torch.no_grad():
        for f, i, name in picks:
            k = f * P + i
            w0 = float(flat[k])
            h = 3e-5 * max(abs(w0), 0.1)
            est = []
            for step in (h, h / 2):
                flat[k] = w0 + step
                lp = float(loss_of(w64))
                flat[k] = w0 - step
                lm = float(loss_of(w64))
                flat[k] = w0
                est.append((lp - lm) / (2 * step))
            noise = NOISE * L0 / (h / 2)
            if abs(est[0] - est[1]) > 1e-6 * abs(est[0]) + 1e-9 * top + 2 * noise:
                rejected += 1           # a ReLU kink inside the step
                continue
            g = float(g_gpu[f, i])
            err = abs(est[0] - g)
            worst = max(worst, err / (abs(g) + 1e-8 * top + noise))
            if err > 1e-6 * abs(g) + 1e-8 * top + noise:
                bad.append((name, f, i, est[0], g))
    print(f"FD on {len(picks)} weights of {len(fields)} fields (loss {L0:.4g}, largest entry {top:.3g}): "
          f"{rejected} at kinks, worst |fd - g| / (|g| + 1e-8 max|g| + noise) = {worst:.3g}")
    assert rejected <= len(picks) // 10
    assert not bad, bad[:5]
    # every tensor is represented among the checked weights
    assert {n for _, _, n in picks} == {n for n, _ in lay}

    # the FP64 GPU gradient against the oracle's analytic FP64 gradient, every weight
    l_ref, g_ref, _ = orc.train_grad(sc, o, d, tgt)
    assert abs(float(loss_of(w64)) - l_ref) <= 1e-12 * l_ref
    errs = block_errors(g_gpu, g_ref, lay, 1e-8)
    print("fp64 worst blocks:", describe(errs))
    assert errs[0][0] <= 1e-8, describe(errs)
    untouched = np.setdiff1d(np.arange(sc.n_fields), fields)
    assert np.all(g_gpu[untouched] == 0.0) and np.all(g_ref[untouched] == 0.0)
    scene.close()


def test_training_subset_gradient_per_tensor(R, orc, subset):
    """The FP32 training-step gradient of the 16-ray subset against the
    oracle: each (field, tensor) block against its own scale (blocks below
    1e-3 of the largest entry against that floor), and entry by entry
    against the oracle's magnitude and kink bound."""
    sc, o, d, tgt, fields = subset
    scene = R.Scene.from_synth(sc)
    loss, grad = R.train_step(scene, _t(o), _t(d), _t(tgt), precision="fp32")
    l_ref, g_ref, _, mag, kin = orc.train_grad(sc, o, d, tgt, magnitude=True, kink=1e-6)
    lay = synth.local_mlp_layout(sc.hidden)
    g = _np(grad)
    errs = block_errors(g, g_ref, lay, 1e-3)
    mb = magnitude_errors(g, g_ref, mag, lay, 2e-4, kin)
    err_all = float(np.abs(g - g_ref).max() / np.abs(g_ref).max())
    print(f"fp32 16-ray subset: loss {float(_np(loss)[0]):.6g} vs {l_ref:.6g}; largest entry "
          f"{np.abs(g_ref).max():.3g}, max error {err_all:.3g} of it; worst blocks: {describe(errs)}; "
          f"against the bound: {describe(mb)}")
    assert abs(float(_np(loss)[0]) - l_ref) <= 1e-5 * l_ref
    assert err_all <= 2e-4
    assert errs[0][0] <= 1e-4, describe(errs)
    assert mb[0][0] <= 1.0, describe(mb)
    scene.close()
