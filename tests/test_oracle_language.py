"""Pins of the language-feature oracle (oracle/language.py) against what the
paper and the mathematics fix: library routines (torch float64 layers,
softmax, cosine similarity and autograd, scipy's cosine distance), closed
forms, limiting cases and finite differences. CPU only."""
import numpy as np
import pytest

import synth
from oracle import decode as D
from oracle import language as LG

torch = pytest.importorskip("torch")


# ------------------------------------------------ decoder of Table 3 and F

def _torch_decoder(x, ws, bs):
    h = torch.from_numpy(D.bf16(x.astype(np.float64)))
    for l, (W, b) in enumerate(zip(ws, bs)):
        h = torch.nn.functional.linear(h, torch.from_numpy(D.bf16(W.astype(np.float64))),
                                       torch.from_numpy(b.astype(np.float64)))
        if l < len(ws) - 1:
            h = torch.from_numpy(D.bf16(torch.relu(h).numpy()))
    return h


@pytest.mark.parametrize("N", [32, 64, 128])
def test_paper_decoder_and_feature_map_match_torch(N):
    """Table 3 decoder (8 -> 128 -> 256 -> N, ReLU between) and F = M S of the
    supplementary inference equations, against torch float64 layers and
    torch.softmax followed by a matrix product."""
    rng = np.random.default_rng(100 + N)
    x = rng.normal(0, 1, (400, 8)).astype(np.float32)
    ws, bs = synth.mlp_init((8, 128, 256, N), 101 + N)
    S = synth.codebook(N, 512, 102 + N)
    r = LG.language_features(x, ws, bs, S)
    z = _torch_decoder(x, ws, bs)
    assert np.allclose(r["logits"], z.numpy(), rtol=1e-12, atol=1e-12)
    Mt = torch.softmax(z, dim=1)
    assert np.allclose(r["M"], Mt.numpy(), rtol=1e-12, atol=1e-15)
    assert np.allclose(r["F"], (Mt @ torch.from_numpy(S.astype(np.float64))).numpy(), rtol=1e-10, atol=1e-14)
    assert np.array_equal(r["top1"], torch.argmax(z, dim=1).numpy())


def test_feature_map_limits():
    """S = identity gives F = M (rows summing to one); a class whose logit
    leads by a wide margin gives F equal to that class's row of S; a constant
    column of S is reproduced in every pixel (F is a convex combination of
    the rows of S)."""
    rng = np.random.default_rng(110)
    N = 64
    x = rng.normal(0, 1, (200, 8)).astype(np.float32)
    ws, bs = synth.mlp_init((8, 128, 256, N), 111)
    r = LG.language_features(x, ws, bs, np.eye(N, dtype=np.float32))
    assert np.allclose(r["F"], r["M"], rtol=0, atol=0)
    assert np.allclose(r["F"].sum(axis=1), 1.0, rtol=0, atol=1e-12)
    S = synth.codebook(N, 96, 112)
    S[:, 5] = 0.25
    b3 = bs[2].copy()
    b3[17] += 200.0
    r2 = LG.language_features(x, ws, bs[:2] + [b3], S)
    assert (r2["top1"] == 17).all()
    assert np.allclose(r2["F"], np.broadcast_to(S[17].astype(np.float64), r2["F"].shape), rtol=0, atol=1e-12)
    r3 = LG.language_features(x, ws, bs, S)
    assert np.allclose(r3["F"][:, 5], 0.25, rtol=0, atol=1e-14)
    assert (np.abs(r3["F"]) <= r3["F_abs"] + 1e-15).all()


def test_rounding_branches():
    """A pixel with no value near a bf16 midpoint has one branch, the oracle's
    logits; an input exactly at a midpoint gives two branches whose inputs
    are the two bf16 neighbours (first-layer logits differ by W1 times one
    bf16 ulp in that input)."""
    rng = np.random.default_rng(140)
    ws, bs = synth.mlp_init((8, 128, 256, 32), 141)
    for _ in range(20):
        x = rng.normal(0, 1, (1, 8)).astype(np.float32)
        fw = D.mlp_forward(x, ws, bs, normalize=False)
        br, ok = D.mlp_branches(x[0], ws, bs, normalize=False)
        assert ok
        if not fw["ambiguous"][0]:
            assert len(br) == 1 and np.array_equal(br[0], fw["logits"][0])
        else:
            assert len(br) >= 2 and any(np.array_equal(b, fw["logits"][0]) for b in br)
    x = np.zeros((1, 8), np.float32)
    x[0, 3] = np.float32(1.0 + 2.0 ** -8)           # halfway between 1 and 1 + 2^-7
    br, ok = D.mlp_branches(x[0], ws[:1], bs[:1], normalize=False)
    assert ok and len(br) == 2
    W = D.bf16(ws[0].astype(np.float64))
    assert np.allclose(np.abs(br[0] - br[1]), np.abs(W[:, 3]) * 2.0 ** -7, rtol=1e-12, atol=0)


# ------------------------------------------------------------ quantisation

def _hybrid(K, N, dc, dd, seed):
    rng = np.random.default_rng(seed)
    S = rng.normal(0, 1, (N, dc + dd))
    F = rng.normal(0, 1, (K, dc + dd))
    return F, S


def test_quantize_distance_matches_scipy_cosine():
    from scipy.spatial.distance import cosine
    F, S = _hybrid(30, 16, 24, 12, 120)
    q = LG.quantize(F, S, 24, lambda_dino=0.5)
    for i, j in [(0, 0), (3, 7), (29, 15), (11, 2)]:
        ref = (1.0 - cosine(F[i, :24], S[j, :24])) + 0.5 * (1.0 - cosine(F[i, 24:], S[j, 24:]))
        assert q["D"][i, j] == pytest.approx(ref, rel=1e-13, abs=1e-14)
    assert np.array_equal(q["m"], np.argmax(q["D"], axis=1))


def test_quantize_codebook_rows_map_to_themselves():
    """Features that are (positively scaled) rows of S quantise to those rows:
    the cosine loss vanishes and r counts how often each row was used."""
    _, S = _hybrid(1, 20, 32, 16, 121)
    idx = np.array([3, 3, 7, 0, 19, 3, 12])
    F = S[idx] * np.array([1.0, 2.0, 0.5, 3.0, 1.0, 0.25, 7.0])[:, None]
    q = LG.quantize(F, S, 32)
    assert np.array_equal(q["m"], idx)
    assert q["L_cos"] == pytest.approx(0.0, abs=1e-14)
    assert np.allclose(q["r"], np.bincount(idx, minlength=20) / len(idx), rtol=0, atol=0)


def test_quantize_dino_part_breaks_clip_ties():
    """Codes 0 and 1 share their CLIP part; the DINO part decides with
    lambda_dino > 0, and the lowest index wins the exact tie at 0."""
    dc, dd = 8, 4
    S = np.zeros((3, dc + dd))
    S[0, :dc] = S[1, :dc] = 1.0
    S[0, dc:] = [1, 0, 0, 0]
    S[1, dc:] = [0, 1, 0, 0]
    S[2, :dc] = -1.0
    S[2, dc:] = [0, 0, 1, 0]
    F = np.concatenate([np.ones((2, dc)), np.array([[0, 1, 0, 0], [0, 2, 0.1, 0]])], axis=1)
    assert (LG.quantize(F, S, dc, lambda_dino=0.5)["m"] == 1).all()
    assert (LG.quantize(F, S, dc, lambda_dino=0.0)["m"] == 0).all()


def test_load_balancing_closed_forms():
    """One shared feature: every index is the same j, r = e_j and
    L_lb = p_j = softmax(D_0)_j. Features orthogonal to every code in both
    parts: D = 0, softmax is uniform, p = 1/N, so L_lb = 1/N whatever r is."""
    F, S = _hybrid(1, 16, 24, 12, 122)
    Fs = np.repeat(F, 50, axis=0)
    q = LG.quantize(Fs, S, 24)
    j = int(q["m"][0])
    e = np.exp(q["D"][0] - q["D"][0].max())
    assert q["L_lb"] == pytest.approx(e[j] / e.sum(), rel=1e-13)
    S2 = np.zeros((5, 6))
    S2[:, 0] = 1.0
    S2[:, 3] = np.arange(1, 6)
    F2 = np.zeros((40, 6))
    F2[:, 1] = 1.0
    F2[:, 4] = np.linspace(1, 2, 40)
    q2 = LG.quantize(F2, S2, 3)
    assert q2["L_lb"] == pytest.approx(1.0 / 5.0, rel=1e-14)
    assert q2["L_cos"] == pytest.approx(1.5, rel=1e-14)     # (1 - 0) + 0.5 (1 - 0)


def _torch_quant_loss(F, St, dc, m, lam_d, lam_cos, lam_lb):
    Ft = torch.from_numpy(F)
    cos = torch.nn.functional.cosine_similarity
    cc = cos(Ft[:, None, :dc], St[None, :, :dc], dim=2, eps=0.0)
    cd = cos(Ft[:, None, dc:], St[None, :, dc:], dim=2, eps=0.0)
    Dm = cc + lam_d * cd
    K, N = Dm.shape
    rows = torch.arange(K)
    mt = torch.from_numpy(m)
    Lcos = ((1 - cc[rows, mt]) + lam_d * (1 - cd[rows, mt])).mean()
    r = torch.bincount(mt, minlength=N).double() / K
    p = torch.softmax(Dm, dim=1).mean(dim=0)
    return lam_cos * Lcos + lam_lb * (r * p).sum()


def test_quantize_gradient_matches_autograd_and_fd():
    """dL_q/dS against torch autograd (cosine_similarity, softmax, the
    argmax held at its value) and against central finite differences of the
    oracle's own L_q (steps that leave every argmax unchanged)."""
    F, S = _hybrid(200, 16, 24, 12, 123)
    q = LG.quantize(F, S, 24, lambda_dino=0.5, lambda_cos=1.0, lambda_lb=0.5)
    St = torch.tensor(S, requires_grad=True)
    L = _torch_quant_loss(F, St, 24, q["m"], 0.5, 1.0, 0.5)
    assert q["L_q"] == pytest.approx(L.item(), rel=1e-13)
    L.backward()
    assert np.allclose(q["grad"], St.grad.numpy(), rtol=1e-10, atol=1e-14)
    rng = np.random.default_rng(124)
    for j, c in zip(rng.integers(0, 16, 12), rng.integers(0, 36, 12)):
        h = 1e-6
        Sp, Sm = S.copy(), S.copy()
        Sp[j, c] += h
        Sm[j, c] -= h
        qp, qm = LG.quantize(F, Sp, 24), LG.quantize(F, Sm, 24)
        assert np.array_equal(qp["m"], q["m"]) and np.array_equal(qm["m"], q["m"])
        assert q["grad"][j, c] == pytest.approx((qp["L_q"] - qm["L_q"]) / (2 * h), rel=1e-6, abs=1e-11)


# -------------------------------------------------------------- smoothing

def test_positional_encoding_closed_form():
    p = np.array([[0.25, -0.5, 1.0]], np.float32)
    assert np.array_equal(LG.positional_encoding(p, 0), p.astype(np.float64))
    e = LG.positional_encoding(p, 2)
    s2 = np.sqrt(0.5)
    ref = [0.25, -0.5, 1.0, s2, -1.0, 0.0, s2, 0.0, -1.0, 1.0, 0.0, 0.0, 0.0, -1.0, 1.0]
    assert np.allclose(e[0], ref, rtol=0, atol=1e-15)


def _torch_smooth(pos, sg, u, ws, bs, w_s, round_bf16):
    Wt = [torch.tensor(D.bf16(W.astype(np.float64)) if round_bf16 else W.astype(np.float64), requires_grad=True)
          for W in ws]
    bt = [torch.tensor(b.astype(np.float64), requires_grad=True) for b in bs]
    sgt = torch.tensor(np.asarray(sg, np.float64), requires_grad=True)
    ut = torch.tensor(np.asarray(u, np.float64), requires_grad=True)
    h = torch.from_numpy(pos.astype(np.float64))
    for l in range(len(ws)):
        h = torch.nn.functional.linear(h, Wt[l], bt[l])
        if l < len(ws) - 1:
            r = torch.relu(h)
            h = r + (torch.from_numpy(D.bf16(r.detach().numpy())) - r).detach() if round_bf16 else r
    s_mlp = h
    t1 = torch.linalg.vector_norm(s_mlp - sgt.detach(), dim=1)
    t2 = torch.clamp(ut.detach(), min=w_s) * torch.linalg.vector_norm(s_mlp.detach() - sgt, dim=1)
    L = (t1 + t2).mean()
    L.backward()
    return L.item(), s_mlp.detach().numpy(), sgt.grad.numpy(), ut.grad, Wt, bt


@pytest.mark.parametrize("round_bf16", [True, False])
def test_smoothing_matches_torch_autograd(round_bf16):
    """Eqs. 13-14 with the stop gradients as torch .detach(): loss, s_MLP,
    dL/ds_G and every MLP gradient; u receives no gradient."""
    rng = np.random.default_rng(130)
    n = 300
    pos = rng.uniform(-4, 4, (n, 3)).astype(np.float32)
    sg = rng.normal(0, 1, (n, 8)).astype(np.float32)
    u = rng.uniform(0, 1, n).astype(np.float32)
    u[:40] = 0.01                                 # below w_s: the floor applies
    ws, bs = synth.mlp_init((3, 128, 128, 128, 8), 131)
    r = LG.smoothing_loss_grad(pos, sg, u, ws, bs, w_s=0.1, round_bf16=round_bf16)
    L, s_mlp, gsg, gu, Wt, bt = _torch_smooth(pos, sg, u, ws, bs, 0.1, round_bf16)
    assert r["loss"] == pytest.approx(L, rel=1e-12)
    assert np.allclose(r["s_mlp"], s_mlp, rtol=1e-12, atol=1e-13)
    assert np.allclose(r["d_sg"], gsg, rtol=1e-10, atol=1e-15)
    assert gu is None or not gu.numpy().any()
    for l in range(4):
        assert np.allclose(r["gW"][l], Wt[l].grad.numpy(), rtol=1e-9, atol=1e-14)
        assert np.allclose(r["gb"][l], bt[l].grad.numpy(), rtol=1e-9, atol=1e-14)


def test_smoothing_closed_forms_and_stop_gradient_routing():
    """s_G = s_MLP: zero loss and zero gradients. One Gaussian: the loss is
    |d| (1 + max(u, w_s)). Finite differences route the gradients: the MLP
    gradient is that of the first term alone (the second term's s_MLP is
    stopped) and the s_G gradient is that of the second term alone (the first
    term's s_G is stopped)."""
    rng = np.random.default_rng(132)
    ws, bs = synth.mlp_init((3, 128, 128, 128, 8), 133)
    pos = rng.uniform(-4, 4, (50, 3)).astype(np.float32)
    out = LG.smooth_forward(pos, ws, bs, round_bf16=False)["out"]
    z = LG.smoothing_loss_grad(pos, out, np.full(50, 0.5), ws, bs, round_bf16=False)
    assert z["loss"] == 0.0 and not z["d_sg"].any() and all(not g.any() for g in z["gW"])
    one = LG.smoothing_loss_grad(pos[:1], out[:1] + np.array([[3.0, 4.0, 0, 0, 0, 0, 0, 0]]), np.array([0.05]),
                                 ws, bs, w_s=0.1, round_bf16=False)
    assert one["loss"] == pytest.approx(5.0 * 1.1, rel=1e-14)
    one = LG.smoothing_loss_grad(pos[:1], out[:1] + np.array([[0, 0, 0, 0, 0, 0, 0, 2.0]]), np.array([0.7]),
                                 ws, bs, w_s=0.1, round_bf16=False)
    assert one["loss"] == pytest.approx(2.0 * 1.7, rel=1e-14)
    sg = rng.normal(0, 1, (50, 8))
    u = rng.uniform(0, 1, 50)
    r = LG.smoothing_loss_grad(pos, sg, u, ws, bs, w_s=0.1, round_bf16=False)

    def first_term(wl):
        o = LG.smooth_forward(pos, wl, bs, round_bf16=False)["out"]
        return np.mean(np.linalg.norm(o - sg, axis=1))

    for l, (i, j) in [(0, (5, 1)), (1, (7, 100)), (2, (127, 3)), (3, (6, 50))]:
        h = 2.0 ** -20            # w +- h stays exact in the float32 masters (|w| < 8)
        wp = [w.copy() for w in ws]
        wm = [w.copy() for w in ws]
        wp[l][i, j] += h
        wm[l][i, j] -= h
        fd = (first_term(wp) - first_term(wm)) / (2 * h)
        assert r["gW"][l][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-12)
    wgt = np.maximum(u, 0.1)
    for g, c in [(0, 0), (10, 7), (49, 3)]:
        h = 1e-6
        sp, sm = sg.copy(), sg.copy()
        sp[g, c] += h
        sm[g, c] -= h
        f2 = lambda s: np.mean(wgt * np.linalg.norm(r["s_mlp"] - s, axis=1))
        assert r["d_sg"][g, c] == pytest.approx((f2(sp) - f2(sm)) / (2 * h), rel=1e-6, abs=1e-12)


def test_smoothing_follows_given_activations():
    """Given its own hidden activations the smoothing loss is unchanged; given
    one activation moved by a bf16 ulp it equals a fresh evaluation of the
    layers above from that activation."""
    rng = np.random.default_rng(134)
    ws, bs = synth.mlp_init((3, 128, 128, 128, 8), 135)
    pos = rng.uniform(-4, 4, (40, 3)).astype(np.float32)
    sg = rng.normal(0, 1, (40, 8))
    u = rng.uniform(0, 1, 40)
    r = LG.smoothing_loss_grad(pos, sg, u, ws, bs)
    r2 = LG.smoothing_loss_grad(pos, sg, u, ws, bs, hidden=r["hs"][1:])
    assert r2["loss"] == r["loss"] and np.array_equal(r2["d_sg"], r["d_sg"])
    assert all(np.array_equal(a, b) for a, b in zip(r["gW"], r2["gW"]))
    hid = [h.copy() for h in r["hs"][1:]]
    g, k = 7, int(np.argmax(hid[2][7]))
    hid[2][g, k] = D.bf16(hid[2][g, k] * (1 + 2.0 ** -7))          # one ulp up
    r3 = LG.smoothing_loss_grad(pos, sg, u, ws, bs, hidden=hid)
    W4 = D.bf16(ws[3].astype(np.float64))
    out = hid[2] @ W4.T + bs[3].astype(np.float64)
    assert np.allclose(r3["s_mlp"], out, rtol=1e-14, atol=1e-14)
    assert not np.allclose(r3["s_mlp"][g], r["s_mlp"][g], rtol=1e-9, atol=0)

