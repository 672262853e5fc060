"""GPU parity of one full optimisation step of the per-Gaussian parameters
(render, L1 + L_u loss, backward, fused Adam with u clamped to [0, 1]) against
the FP64 oracle, through the C ABI.

Sec. 3.1 Eq. 1 (renderer), Sec. 3.4.2 Eq. 11 (L_u), Sec. 4 (Adam, lr 1e-3,
betas (0.9, 0.999)).
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import decode as D
from oracle import oracle as O
from tests import parity as PT

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def check_training_step(scene, cams, o, d_sem, target, clamp_checked):
    """One TrainStep against the oracle: forward (ambiguity rule), loss and
    dL/dout, every per-Gaussian gradient along the GPU's branches, Adam's
    moments and the update (u clamped to [0, 1])."""
    from paper_2311_18482_amd.train import TrainStep, GROUPS
    C = scene.n_channels
    oo = PT.oracle_opts(o)
    params = {k: v.clone() for k, v in PT.to_dev(scene).items()}
    p0 = {k: params[k].cpu().numpy().astype(np.float64) for k in GROUPS}
    ts = TrainStep(cams, params, torch.from_numpy(target).cuda(), d_sem, o=o, lambda_u=1.0, lr=1e-3)
    note(f"one training step: n={scene.n} views={len(cams)} C={C} tile={o.tile} batch={o.lds_batch}")
    ts.step()
    torch.cuda.synchronize()
    assert not ts.overflowed()
    # forward and loss
    fwd = O.forward(scene, cams, oo)
    masks, stats = PT.compare_render(ts.out, ts.T, ts.last, scene, cams, oo, fwd)
    out_ref = np.concatenate([v["out"].reshape(-1) for v in fwd["views"]])
    loss_ref, G_ref = D.l1_loss_grad(out_ref, target, cams, C, d_sem, lambda_u=1.0)
    assert ts.loss.item() == pytest.approx(loss_ref, rel=2e-5)
    d_out = ts.d_out.cpu().numpy().astype(np.float64)
    # dL/dout: sign(out - target) / count, except where the rendered value is
    # within float32 distance of its target (either sign is then correct)
    near = np.abs(out_ref - target.astype(np.float64)) < 1e-5
    assert np.allclose(d_out[~near], G_ref[~near], rtol=1e-6, atol=0)     # float32 1 / count
    note(f"render {stats}; {int(near.sum())} loss elements at their target")
    del out_ref, G_ref
    # gradients: the oracle backward of the same dL/dout, along the GPU's branches
    ref = O.backward(scene, cams, oo, fwd, d_out, flip_masks=masks, magnitudes=True, mag_cond=PT.MAG_COND)
    del fwd
    # Adam's first step from zero moments: m = (1 - b1) g, v = (1 - b2) g^2,
    # p -= lr g / (|g| + eps), then u clamped to [0, 1]
    got_g = {k: ts.g[k].cpu().numpy().astype(np.float64) for k in GROUPS}
    worst = PT.compare_grads(got_g, ref, scene.n, mag=ref["mag"])
    for k in GROUPS:
        g = ref[k].reshape(p0[k].shape)
        m = ts.m[k].cpu().numpy().astype(np.float64)
        v = ts.v[k].cpu().numpy().astype(np.float64)
        assert np.allclose(m, 0.1 * got_g[k].reshape(m.shape), rtol=1e-6, atol=1e-30), k
        assert np.allclose(v, 1e-3 * got_g[k].reshape(v.shape) ** 2, rtol=1e-5, atol=1e-30), k
        p1_ref, _, _ = D.adam(p0[k], g, np.zeros_like(g), np.zeros_like(g), 1)
        if k == "channels":
            p1_ref[:, C - 1] = np.clip(p1_ref[:, C - 1], 0.0, 1.0)
        p1 = params[k].cpu().numpy().astype(np.float64)
        # entries with a clear gradient move by lr * sign(g); the others by less
        scale = np.abs(g).max()
        clear = np.abs(g) > 1e-4 * scale
        assert np.allclose(p1[clear], p1_ref[clear], rtol=0, atol=2e-6), k
        # at most lr, plus the float32 rounding of the stored parameter (one
        # spacing of the stored value bounds the half ulp of either rounding)
        ulp = np.spacing(np.abs(p1).astype(np.float32)).astype(np.float64)
        assert (np.abs(p1 - p0[k]) <= 1e-3 * (1 + 1e-5) + ulp + 1e-12).all(), k
    u = params["channels"][:, C - 1].cpu().numpy()
    assert (u >= 0.0).all() and (u <= 1.0).all()
    if clamp_checked:
        blended = np.abs(ref["channels"]).sum(axis=1) > 0
        assert (u[:200][blended[:200]] == 0.0).sum() >= 20
    note(f"gradient worst ratios { {k: round(w['ratio'], 4) for k, w in worst.items()} }")


def test_training_step_matches_oracle():
    from paper_2311_18482_amd import raster as R
    d_sem = 16
    scene = synth.make_scene(8000, 55, synth.VOL_C1, d_sem=d_sem)
    C = scene.n_channels
    assert C == 20
    scene.channels[:200, C - 1] = 0.0005          # L_u pushes u down: Adam crosses 0, the clamp holds it
    cams = [synth.camera_front(128, 96, 128.0)]
    R2, t2 = synth.look_at((1.5, -1.0, -2.0), target=(0.0, 0.0, 4.0))
    cams.append(synth.Camera(96, 80, 90.0, 90.0, 48.0, 40.0, R2, t2))
    target = synth.targets_l1(cams, C, d_sem, 56)
    check_training_step(scene, cams, R.opts(tile=16, lds_batch=128), d_sem, target, True)


@pytest.mark.timeout(1500)
def test_training_step_at_c5_size():
    """The full training step as the bench times it: 3M Gaussians with RGB,
    a 16-d semantic feature and u, four 1920x1080 views, 32-pixel tiles, LDS
    batch 256, ids-only lists."""
    from paper_2311_18482_amd import raster as R
    scene, cams = synth.workload_c5()
    d_sem = 16
    target = synth.targets_l1(cams, scene.n_channels, d_sem, 205)
    check_training_step(scene, cams, R.opts(tile=32, lds_batch=256, ids_only=True), d_sem, target, False)
