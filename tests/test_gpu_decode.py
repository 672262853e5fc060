"""GPU parity of decoding, decoder training, Adam and the training-step loss
against the FP64 oracle, through the C ABI.

Plain decode: Sec. 3.3 Eq. 4 (cosine max-similarity over S); learned decode:
Eq. 8 and the supplementary inference equation; training: Eq. 9 with Adam
(Sec. 4); loss: per-view L1 plus the L_u regulariser of Eq. 11.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import decode as D
from tests import parity as PT

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_18482_amd import raster
    assert torch.cuda.is_available()
    return raster.Context(0)


@pytest.fixture(scope="module")
def DEC():
    from paper_2311_18482_amd import decode
    return decode


def features(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.normal(0, 1, (n, 8)).astype(np.float32)
    f[: n // 20] *= rng.uniform(0, 0.05, (n // 20, 1)).astype(np.float32)   # near-transparent pixels
    f[0] = 0.0
    return f


def check_top1(top_g, score_ref, top_ref, rel_margin):
    s = np.sort(score_ref, axis=1)
    gap = s[:, -1] - s[:, -2]
    clear = gap > rel_margin * np.maximum(np.abs(s[:, -1]), 1e-30)
    assert np.array_equal(top_g[clear], top_ref[clear]), int((top_g[clear] != top_ref[clear]).sum())
    return int((~clear).sum())


@pytest.mark.parametrize("K,Dm", [(128, 512), (64, 256), (32, 64)])
def test_plain_and_folded_decode(ctx, DEC, K, Dm):
    n = 9001                                                      # ragged final tile
    f = features(n, 1 + K)
    Pm = synth.projection(Dm, 8, 9)
    Cb = synth.codebook(K, Dm, 10)
    probs_ref, top_ref = D.decode_plain(f, Pm, Cb)
    z = f.astype(np.float64) @ Pm.astype(np.float64).T
    cos = (z @ Cb.astype(np.float64).T) / np.maximum(np.linalg.norm(z, axis=1, keepdims=True), 1e-300)
    fd_ = torch.from_numpy(f).cuda()
    Pd, Cd = torch.from_numpy(Pm).cuda(), torch.from_numpy(Cb).cuda()
    # row-major [P][8] and planar [8][P] inputs
    for feat in (DEC.rowmajor_features(fd_), (fd_.t().contiguous(), n, n, 1)):
        top, pr = DEC.decode_plain(ctx, feat, Pd, Cd, probs=True)
        torch.cuda.synchronize()
        amb = check_top1(top.cpu().numpy(), cos, top_ref, 1e-5)
        assert amb < n // 100
        assert np.abs(pr.cpu().numpy() - probs_ref).max() < 1e-5
        assert top[0].item() == 0
    folded = DEC.decode_fold(ctx, Pd, Cd)
    top, pr = DEC.decode_folded(ctx, DEC.rowmajor_features(fd_), folded, K, probs=True)
    torch.cuda.synchronize()
    check_top1(top.cpu().numpy(), cos, top_ref, 1e-5)
    assert np.abs(pr.cpu().numpy() - probs_ref).max() < 1e-5


@pytest.mark.parametrize("K,normalize", [(128, True), (64, True), (32, True), (128, False)])
def test_mlp_decode(ctx, DEC, K, normalize):
    n = 5000 + 17
    f = features(n, 20 + K)
    ws, bs = synth.mlp_init((8, 64, 64, K), 30 + K)
    note(f"decode_mlp K={K} normalize={normalize}")
    params = DEC.mlp_pack(ws, bs).cuda()
    top, pr = DEC.decode_mlp(ctx, DEC.rowmajor_features(torch.from_numpy(f).cuda()), params, K, probs=True,
                             normalize=normalize)
    torch.cuda.synchronize()
    # the top-1-only kernel (logits consumed block by block), row-major and planar input
    fd_ = torch.from_numpy(f).cuda()
    top_r, _ = DEC.decode_mlp(ctx, DEC.rowmajor_features(fd_), params, K, normalize=normalize)
    top_p, _ = DEC.decode_mlp(ctx, (fd_.t().contiguous(), n, n, 1), params, K, normalize=normalize)
    torch.cuda.synchronize()
    top, pr = top.cpu().numpy(), pr.cpu().numpy()
    assert np.array_equal(top_r.cpu().numpy(), top) and np.array_equal(top_p.cpu().numpy(), top)
    # pixels with no bf16 rounding near a midpoint: the oracle's own forward;
    # the others: the oracle branch whose roundings the kernel took
    logits, resolved, n_amb = PT.check_mlp_probs(pr.astype(np.float64), f, ws, bs, normalize)
    assert n_amb < n // 2, n_amb
    s = np.sort(logits, axis=1)
    clear = resolved & ((s[:, -1] - s[:, -2]) > 1e-4 * (np.abs(s[:, -1]) + 1))
    assert np.array_equal(top[clear], np.argmax(logits, axis=1)[clear])
    assert clear.mean() > 0.99, clear.mean()
    note(f"ambiguous pixels {n_amb}, resolved {int(resolved.sum())} of {n}")


def test_decodes_at_bench_size(ctx, DEC):
    """The decodes the bench times, at its size (32 views of 1920x1080 8-d
    features: 66.4M pixels, K = 128, codebook 128 x 512, projection 512 x 8)
    in the same launches (top-1 only): the learned decode with normalised and
    raw input, the direct and the folded plain decode. 4000 sampled pixels
    (the first, the ragged last 40, random ones) against the oracle: the
    plain decodes' top-1 outside a 1e-5 cosine margin; the learned decode's
    top-1 is the oracle's argmax where no bf16 value lies near a rounding
    midpoint (outside a 1e-4 logit margin), and elsewhere the argmax of one
    of the pixel's rounding branches."""
    P, K, Dm = 32 * 1920 * 1080, 128, 512
    f = features(P, 80)
    ws, bs = synth.mlp_init((8, 64, 64, K), 81)
    Pm = synth.projection(Dm, 8, 82)
    Cb = synth.codebook(K, Dm, 83)
    fd_ = torch.from_numpy(f).cuda()
    params = DEC.mlp_pack(ws, bs).cuda()
    Pd, Cd = torch.from_numpy(Pm).cuda(), torch.from_numpy(Cb).cuda()
    note(f"decodes at P={P} K={K}")
    fr = DEC.rowmajor_features(fd_)
    tops = {}
    for normalize in (True, False):
        t, _ = DEC.decode_mlp(ctx, fr, params, K, normalize=normalize)
        tops[normalize] = t
    t_plain, _ = DEC.decode_plain(ctx, fr, Pd, Cd)
    t_fold, _ = DEC.decode_folded(ctx, fr, DEC.decode_fold(ctx, Pd, Cd), K)
    torch.cuda.synchronize()
    rng = np.random.default_rng(84)
    idx = np.unique(np.concatenate([[0], np.arange(P - 40, P), rng.integers(0, P, 4000)]))
    it = torch.from_numpy(idx).cuda()
    fs = f[idx]
    # plain decodes
    _, top_ref = D.decode_plain(fs, Pm, Cb)
    z = fs.astype(np.float64) @ Pm.astype(np.float64).T
    cos = (z @ Cb.astype(np.float64).T) / np.maximum(np.linalg.norm(z, axis=1, keepdims=True), 1e-300)
    for t in (t_plain, t_fold):
        amb = check_top1(t[it].cpu().numpy(), cos, top_ref, 1e-5)
        assert amb < len(idx) // 100
    # learned decodes
    for normalize, t in tops.items():
        tg = t[it].cpu().numpy()
        fw = D.mlp_forward(fs, ws, bs, normalize=normalize)
        s = np.sort(fw["logits"], axis=1)
        clear = ~fw["ambiguous"] & ((s[:, -1] - s[:, -2]) > 1e-4 * (np.abs(s[:, -1]) + 1))
        assert np.array_equal(tg[clear], np.argmax(fw["logits"], axis=1)[clear])
        assert clear.mean() > 0.9, clear.mean()
        for i in np.nonzero(fw["ambiguous"])[0]:
            br, complete = D.mlp_branches(fs[i], ws, bs, normalize=normalize)
            if complete:
                assert tg[i] in {int(np.argmax(b)) for b in br}, i
        note(f"normalize={normalize}: ambiguous {int(fw['ambiguous'].sum())} of {len(idx)} sampled")


@pytest.mark.parametrize("normalize", [True, False])
def test_mlp_gradient_and_train_step(ctx, DEC, normalize):
    K, B = 128, 6000
    f = features(B, 40)
    rng = np.random.default_rng(41)
    y = rng.integers(0, K, B).astype(np.int32)
    ws, bs = synth.mlp_init((8, 64, 64, K), 42)
    note(f"mlp train K={K} B={B} normalize={normalize}")
    tr = DEC.MlpTrainer(ctx, DEC.mlp_pack(ws, bs), K, B, normalize=normalize)
    fd_ = torch.from_numpy(f).cuda()
    yd = torch.from_numpy(y).cuda()
    grad, loss = tr.grad_only(DEC.rowmajor_features(fd_), yd)
    # the training forward is the decoder's: its probabilities name the
    # rounding branch each pixel took, and the oracle's gradient follows the
    # oracle's activations of that branch
    _, pr = DEC.decode_mlp(ctx, DEC.rowmajor_features(fd_), tr.params, K, probs=True, normalize=normalize)
    torch.cuda.synchronize()
    hid = []
    _, resolved, n_amb = PT.check_mlp_probs(pr.cpu().numpy().astype(np.float64), f, ws, bs, normalize,
                                            hidden_out=hid)
    loss_ref, gW, gb = D.mlp_grads(f, y, ws, bs, normalize=normalize, hidden=hid)
    g = grad.cpu().numpy().astype(np.float64)
    ref = np.concatenate([np.concatenate([w.reshape(-1), b]) for w, b in zip(gW, gb)])
    assert abs(loss.item() - loss_ref) < 1e-6 * abs(loss_ref), (loss.item(), loss_ref)
    # float32 sums of split-bf16 (16 significant bits) upstream gradients
    # times exact bf16 operands: each segment within 3e-5 of its norm
    off, worst = 0, 0.0
    for w, b in zip(gW, gb):
        for part in (w.reshape(-1), b):
            seg = g[off:off + part.size]
            r = np.linalg.norm(seg - part) / np.linalg.norm(part)
            worst = max(worst, r)
            assert r <= 3e-5, (off, r)
            off += part.size
    assert off == g.size
    note(f"ambiguous {n_amb}, resolved {int(resolved.sum())} of {B}; worst segment error {worst:.2e}")
    # one full step (gradient + Adam) vs the oracle's Adam on the oracle gradient
    p0 = DEC.mlp_pack(ws, bs).numpy().astype(np.float64)
    tr.step(DEC.rowmajor_features(fd_), yd)
    torch.cuda.synchronize()
    p1_ref, _, _ = D.adam(p0, ref, np.zeros_like(p0), np.zeros_like(p0), 1)
    p1 = tr.params.cpu().numpy().astype(np.float64)
    # first Adam step moves each weight by ~lr * sign(g); compare the moves
    moved = np.abs(ref) > 1e-4 * np.abs(ref).max()
    assert np.allclose(p1[moved], p1_ref[moved], rtol=0, atol=2e-6)


def test_adam_groups_and_clamp(ctx, DEC):
    """Groups of one and several workgroup chunks, an empty one, ragged tails;
    16-byte aligned groups take the kernel's four-element path, the last one
    (every array one element off alignment) its element path; clamps whose
    period is shorter and longer than four."""
    rng = np.random.default_rng(50)
    sizes = [1000, 37, 4096 * 5, 0, 4096 * 2 + 3]
    host = [dict(p=rng.normal(0, 1, n), m=np.zeros(n), v=np.zeros(n)) for n in sizes]

    def buf(n, off, x=None):
        b = torch.zeros(n + off, dtype=torch.float32, device="cuda")[off:]
        if x is not None:
            b.copy_(torch.tensor(x, dtype=torch.float32))
        return b
    dev = [dict(param=buf(n, off, h["p"]), m=buf(n, off), v=buf(n, off), grad=buf(n, off))
           for h, n, off in zip(host, sizes, [0, 0, 0, 0, 1])]
    clamps = {0: (3, 2, -0.2, 0.2), 2: (5, 4, 0.0, 1.0), 4: (7, 0, -0.5, 0.5)}
    for k, c in clamps.items():
        dev[k]["clamp"] = c                        # every c[0]-th column from c[1] clamped to [c[2], c[3]]
    for step in range(1, 5):
        for h, d in zip(host, dev):
            g = rng.normal(0, 1, h["p"].size).astype(np.float32)
            d["grad"].copy_(torch.from_numpy(g))
            h["p"], h["m"], h["v"] = D.adam(h["p"], g.astype(np.float64), h["m"], h["v"], step,
                                            lr=1e-2)
        for k, (every, off, lo, hi) in clamps.items():
            host[k]["p"][off::every] = np.clip(host[k]["p"][off::every], lo, hi)
        DEC.adam(ctx, dev, step, lr=1e-2)
    torch.cuda.synchronize()
    for h, d in zip(host, dev):
        got = d["param"].cpu().numpy().astype(np.float64)
        assert np.allclose(got, h["p"], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("sizes", [((37, 21), (64, 48)), ((32, 16), (64, 48)), ((32, 16), (37, 21), (16, 8))])
def test_l1_loss_gradient(ctx, DEC, sizes):
    """Unaligned planes (odd pixel counts) take the kernel's element path,
    16-byte aligned ones its four-element path, a mix both."""
    from paper_2311_18482_amd import raster as R
    cams = [synth.camera_front(w, h, float(w)) for w, h in sizes]
    C, ds = 20, 16
    rng = np.random.default_rng(60)
    total = sum(C * c.width * c.height for c in cams)
    out = rng.normal(0, 1, total).astype(np.float32)
    tgt = synth.targets_l1(cams, C, ds, 61)
    loss_ref, g_ref = D.l1_loss_grad(out, tgt, cams, C, ds, lambda_u=1.0)
    views = R.views_build(cams, R.opts(), ctx.device)
    d_out, loss = DEC.l1_loss_grad(ctx, torch.from_numpy(out).cuda(), torch.from_numpy(tgt).cuda(),
                                   views, C, 3 + ds, 1.0)
    torch.cuda.synchronize()
    assert np.allclose(d_out.cpu().numpy(), g_ref, rtol=1e-6, atol=1e-12)
    assert loss.item() == pytest.approx(loss_ref, rel=1e-5)
