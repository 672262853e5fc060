"""GPU parity of the adaptive spatial smoothing of Sec. 3.4.2 (Eqs. 13-14,
PE and MLP of Table 4) against the FP64 oracle, through the C ABI: the bf16
hidden activations, the loss, dL/ds_G and every MLP gradient."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import decode as D
from oracle import language as LG

pytestmark = pytest.mark.gpu


def kappa(n):
    """Error allowance of the weight-gradient sums in units of sum |term|:
    float32 sums within a workgroup's chunk of 4096 Gaussians and the 16-bit
    split of dz (3e-5), plus one float32 atomic per chunk."""
    return 3e-5 + -(-n // 4096) * 2.0 ** -24


def note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_18482_amd import raster
    assert torch.cuda.is_available()
    return raster.Context(0)


def planes(ws, n, Gp):
    """The bf16 hidden activations h1, h2, h3 from the workspace: after the
    16-row input plane, three 128-row planes in the weight gradient's operand
    order ([Gp / 16 steps][4 row blocks][2 Gaussian halves][32 rows][8
    Gaussians]: row 32 b + r, Gaussian 16 s + 8 k + e). Returned [n][128]."""
    b = ws.view(torch.bfloat16)
    out = []
    for k in range(3):
        off = 16 * Gp + k * 128 * Gp
        f = b[off:off + 128 * Gp].view(Gp // 16, 4, 2, 32, 8)
        out.append(f.permute(0, 2, 4, 1, 3).reshape(Gp, 128)[:n].float().cpu().numpy().astype(np.float64))
    return out


def check_activations(pos, ws, bs, hid):
    """Each GPU activation is the oracle's bf16(relu(z)) of the GPU's previous
    layer, up to float32 accumulation error in z: rounding is monotone, so the
    activation lies between the roundings of relu at z - e and z + e, with e
    bounding the float32 error of the sum. Where those two agree it is exact."""
    h = LG.positional_encoding(pos, 0)
    n_amb = 0
    for l in range(3):
        W = D.bf16(ws[l].astype(np.float64))
        b = bs[l].astype(np.float64)
        z = h @ W.T + b
        e = 2e-6 * (np.abs(h) @ np.abs(W).T + np.abs(b))
        lo, hi = D.bf16(np.maximum(z - e, 0.0)), D.bf16(np.maximum(z + e, 0.0))
        exp = D.bf16(np.maximum(z, 0.0))
        ok = (hid[l] >= lo) & (hid[l] <= hi)
        bad = np.argwhere(~ok)[:5]
        assert ok.all(), (l, int((~ok).sum()), [(tuple(i), hid[l][tuple(i)], lo[tuple(i)], hi[tuple(i)], z[tuple(i)])
                                                 for i in bad])
        n_amb += int((hid[l] != exp).sum())
        h = hid[l]
    return n_amb


@pytest.mark.parametrize("n", [20000 + 13, 777, 1_000_000])
def test_smoothing_matches_oracle(ctx, n):
    """The last size is the bench's (the 1M Gaussians of the 1080p scene), in
    its launch configuration."""
    from paper_2311_18482_amd import decode as DEC
    rng = np.random.default_rng(180 + n)
    C, sem, uch = 12, 3, 11
    pos = rng.uniform(-4, 4, (n, 3)).astype(np.float32)
    chans = rng.normal(0, 0.3, (n, C)).astype(np.float32)
    chans[:, uch] = rng.uniform(0, 1, n)
    chans[: n // 10, uch] = 0.02                              # below w_s: the floor applies
    ws, bs = synth.mlp_init((3, 128, 128, 128, 8), 181)
    params = torch.cat([torch.from_numpy(np.concatenate([W.reshape(-1), b])) for W, b in zip(ws, bs)]).cuda()
    assert params.numel() == DEC.smooth_param_count()
    lam = 0.7
    d0 = rng.normal(0, 1e-3, (n, C)).astype(np.float32)
    d_ch = torch.from_numpy(d0).cuda()
    grad = torch.zeros_like(params)
    loss = torch.zeros(1, device="cuda")
    note(f"smoothing n={n}")
    wsp = DEC.smooth_loss_grad(ctx, torch.from_numpy(pos).cuda(), torch.from_numpy(chans).cuda(), sem, uch, params,
                               grad, d_ch, loss, w_s=0.1, lambda_smo=lam)
    torch.cuda.synchronize()
    Gp = (n + 63) // 64 * 64
    hid = planes(wsp, n, Gp)
    n_amb = check_activations(pos, ws, bs, hid)
    # everything else along the GPU's activations
    sg, u = chans[:, sem:sem + 8], chans[:, uch]
    r = LG.smoothing_loss_grad(pos, sg, u, ws, bs, w_s=0.1, hidden=hid)
    # the loss is one float32 atomic per wave (64 Gaussians): a random walk of
    # about sqrt(n / 64) roundings of 2^-24 (under 1e-5 up to ~1e5 Gaussians)
    assert loss.item() == pytest.approx(lam * r["loss"], rel=1e-5 + 4.0 * np.sqrt(n / 64) * 2.0 ** -24)
    after = d_ch.cpu().numpy().astype(np.float64)
    dch = after - d0
    # the accumulated channel gradient is stored in float32: 2^-24 of the sum per element
    store = 2.0 ** -24 * np.linalg.norm(after[:, sem:sem + 8], axis=1)
    others = np.delete(np.arange(C), np.arange(sem, sem + 8))
    assert not dch[:, others].any()                           # u and RGB get nothing
    # s_MLP in float32: |error| <= 1e-5 sum |W4| |h3| per output; the unit vector
    # (s_MLP - s_G) / |.| then moves by at most 2 |error| / |.|
    W4 = D.bf16(ws[3].astype(np.float64))
    smag = np.linalg.norm(hid[2] @ np.abs(W4).T + np.abs(bs[3]), axis=1)
    wgt = np.maximum(u, 0.1)
    du = np.minimum(2.0, 2e-5 * smag / np.maximum(r["norm"], 1e-30))
    err = np.linalg.norm(dch[:, sem:sem + 8] - lam * r["d_sg"], axis=1)
    assert (err <= lam * wgt / n * du + 1e-6 * lam * wgt / n + store).all()
    # MLP gradients: errors of dz4 (as above) carried down the layers, plus
    # kappa(n) sum |term| of each product
    g = grad.cpu().numpy().astype(np.float64)
    Wb = [D.bf16(w.astype(np.float64)) for w in ws]
    e = (lam / n * du)[:, None] * np.ones((1, 8))             # |error| of dz4 per Gaussian and output
    dz = lam * np.abs(r["d_sg"]) / np.maximum(wgt, 1e-30)[:, None]   # |dz4| = lam |unit| / n
    hs = r["hs"]
    sizes = [(128, 3), (128, 128), (128, 128), (8, 128)]
    offs = np.cumsum([0] + [a * b_ + a for a, b_ in sizes])
    for l in range(3, -1, -1):
        gW = g[offs[l]:offs[l] + sizes[l][0] * sizes[l][1]].reshape(sizes[l])
        gb = g[offs[l] + sizes[l][0] * sizes[l][1]:offs[l + 1]]
        bound = e.T @ np.abs(hs[l]) + kappa(n) * (dz.T @ np.abs(hs[l])) + 1e-12
        assert (np.abs(gW - lam * r["gW"][l]) <= bound).all(), (l, float((np.abs(gW - lam * r["gW"][l]) / bound).max()))
        bb = e.sum(axis=0) + kappa(n) * dz.sum(axis=0) + 1e-12
        assert (np.abs(gb - lam * r["gb"][l]) <= bb).all(), (l, float((np.abs(gb - lam * r["gb"][l]) / bb).max()))
        if l > 0:
            gate = hs[l] > 0
            e = (e @ np.abs(Wb[l])) * gate + 3e-5 * (dz @ np.abs(Wb[l])) * gate
            dz = (dz @ np.abs(Wb[l])) * gate
    note(f"n={n}: loss {loss.item():.6g} vs {lam * r['loss']:.6g}, activations off the oracle's by rounding: {n_amb}")
