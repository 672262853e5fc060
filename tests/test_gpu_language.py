"""GPU parity of the language-feature path against the FP64 oracle, through
the C ABI: the decoder of Table 3 (8 -> 128 -> 256 -> N, M_infer =
softmax(D_MLP(R_s))) and the language feature map F = M_infer S of the
supplementary inference equations."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import decode as D
from oracle import language as LG
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


def features(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.normal(0, 1, (n, 8)).astype(np.float32)
    f[: n // 20] *= rng.uniform(0, 0.05, (n // 20, 1)).astype(np.float32)
    f[0] = 0.0
    return f


@pytest.mark.parametrize("N,normalize", [(128, False), (64, False), (32, False), (128, True)])
def test_paper_decoder_matches_oracle(ctx, N, normalize):
    from paper_2311_18482_amd import decode as DEC
    n = 6000 + 29                                            # ragged final tile
    f = features(n, 150 + N)
    ws, bs = synth.mlp_init((8, 128, 256, N), 151 + N)
    params = DEC.mlp_pack(ws, bs).cuda()
    assert params.numel() == DEC.dmlp_param_count(N)
    fd = torch.from_numpy(f).cuda()
    note(f"decode_dmlp N={N} normalize={normalize} P={n}")
    t1, pr, p16 = DEC.decode_dmlp(ctx, DEC.rowmajor_features(fd), params, N, probs=True, probs_f16=True,
                                  normalize=normalize)
    t_only, _, _ = DEC.decode_dmlp(ctx, DEC.rowmajor_features(fd), params, N, normalize=normalize)
    t_planar, _, _ = DEC.decode_dmlp(ctx, (fd.t().contiguous(), n, n, 1), params, N, normalize=normalize)
    torch.cuda.synchronize()
    # one kernel writes both precisions from the same float32 probability
    assert torch.equal(p16, pr.half())
    t1, pr = t1.cpu().numpy(), pr.cpu().numpy().astype(np.float64)
    assert np.array_equal(t_only.cpu().numpy(), t1) and np.array_equal(t_planar.cpu().numpy(), t1)
    logits, resolved, n_amb = PT.check_mlp_probs(pr, f, ws, bs, normalize)
    s = np.sort(logits, axis=1)
    clear = resolved & ((s[:, -1] - s[:, -2]) > 1e-4 * (np.abs(s[:, -1]) + 1))
    assert np.array_equal(t1[clear], np.argmax(logits, axis=1)[clear])
    note(f"ambiguous pixels {n_amb}, resolved {int(resolved.sum())} of {n}")


@pytest.mark.parametrize("N,d,out_f16,n,misalign", [(128, 512, False, 3007, 0), (32, 544, False, 3007, 0),
                                                    (64, 96, True, 3007, 0), (128, 544, True, 3010, 0),
                                                    (64, 96, False, 3010, 0), (128, 512, True, 3010, 1),
                                                    (32, 4096, True, 1030, 0)])
def test_language_features_match_oracle(ctx, N, d, out_f16, n, misalign):
    """F = M S: against the float64 product of the very half-precision inputs
    the kernel read (float32 accumulation is the only rounding: within
    gamma_N of M |S|), and against the oracle's exact M S (the half roundings
    of M and S add at most 2^-10 of M |S|, plus 2^-25 |S| per class where a
    probability is subnormal in half precision). An even pixel count with F
    16-byte aligned takes the kernel's paired-pixel stores, an odd one or an F
    one element off alignment its element stores (ragged last group either
    way)."""
    from paper_2311_18482_amd import decode as DEC
    f = features(n, 160 + d)
    ws, bs = synth.mlp_init((8, 128, 256, N), 161 + N)
    S = synth.codebook(N, d, 162 + d)
    params = DEC.mlp_pack(ws, bs).cuda()
    note(f"language_features N={N} d={d} out_f16={out_f16} n={n} misalign={misalign}")
    _, pr, p16 = DEC.decode_dmlp(ctx, DEC.rowmajor_features(torch.from_numpy(f).cuda()), params, N, probs=True,
                                 probs_f16=True, top1=False)
    buf = torch.full((d * n + misalign,), float("nan"), dtype=torch.float16 if out_f16 else torch.float32,
                     device="cuda")
    Fg = DEC.language_features(ctx, p16, torch.from_numpy(S).cuda(), out_f16=out_f16,
                               F=buf[misalign:].view(d, n))
    torch.cuda.synchronize()
    assert Fg.shape == (d, n)
    Fg = Fg.float().cpu().numpy().astype(np.float64).T
    M16 = p16.float().cpu().numpy().astype(np.float64)
    S16 = S.astype(np.float16).astype(np.float64)
    ref = M16 @ S16
    ref_abs = M16 @ np.abs(S16)
    bound = N * 2.0 ** -24 * ref_abs + (2.0 ** -11 * np.abs(ref) + 2.0 ** -25 if out_f16 else 1e-30)
    assert (np.abs(Fg - ref) <= bound).all(), float((np.abs(Fg - ref) / bound).max())
    # end to end against the oracle (non-ambiguous pixels of the decoder)
    o = LG.language_features(f, ws, bs, S)
    amb = o["ambiguous"]
    tol = (2.0 ** -10 + 2e-5) * o["F_abs"] + N * 2.0 ** -25 * np.abs(S).max() + (bound if out_f16 else 0.0)
    assert (np.abs(Fg - o["F"])[~amb] <= tol[~amb]).all()
    note(f"max rel err vs exact {float((np.abs(Fg - o['F']) / np.maximum(o['F_abs'], 1e-30))[~amb].max()):.3g}")


def test_paper_decoder_and_features_at_bench_size(ctx):
    """The Table 3 decoder and F = M S at the size the bench times them (four
    1920x1080 views of 8-d rendered features, N = 128, d = 512, float32 F),
    in the same launch configurations: both decode kernels agree on every
    pixel's top-1, both precisions come from one probability, and 4000
    sampled pixels (the first, the ragged last 40, random ones) match the
    oracle: the decoder by rounding-branch replay, their F columns within the
    bounds of the small-size test."""
    from paper_2311_18482_amd import decode as DEC
    P, N, d = 4 * 1920 * 1080, 128, 512
    f = features(P, 190)
    ws, bs = synth.mlp_init((8, 128, 256, N), 191)
    S = synth.codebook(N, d, 192)
    params = DEC.mlp_pack(ws, bs).cuda()
    fd = torch.from_numpy(f).cuda()
    note(f"decode_dmlp + language_features at P={P} N={N} d={d}")
    t_only, _, _ = DEC.decode_dmlp(ctx, DEC.rowmajor_features(fd), params, N)
    t1, pr, p16 = DEC.decode_dmlp(ctx, DEC.rowmajor_features(fd), params, N, probs=True, probs_f16=True)
    Fg = DEC.language_features(ctx, p16, torch.from_numpy(S).cuda())
    Fh = DEC.language_features(ctx, p16, torch.from_numpy(S).cuda(), out_f16=True)
    torch.cuda.synchronize()
    assert torch.equal(t_only, t1)
    assert torch.equal(p16, pr.half())
    # the half map is the same float32 sums rounded to nearest
    assert torch.equal(Fh, Fg.half())
    del Fh
    rng = np.random.default_rng(193)
    idx = np.unique(np.concatenate([[0], np.arange(P - 40, P), rng.integers(0, P, 4000)]))
    it = torch.from_numpy(idx).cuda()
    prs = pr[it].cpu().numpy().astype(np.float64)
    t1s = t1[it].cpu().numpy()
    Fs = Fg[:, it].t().cpu().numpy().astype(np.float64)
    M16 = p16[it].float().cpu().numpy().astype(np.float64)
    del pr, p16, Fg
    logits, resolved, n_amb = PT.check_mlp_probs(prs, f[idx], ws, bs, False)
    s = np.sort(logits, axis=1)
    clear = resolved & ((s[:, -1] - s[:, -2]) > 1e-4 * (np.abs(s[:, -1]) + 1))
    assert np.array_equal(t1s[clear], np.argmax(logits, axis=1)[clear])
    assert clear.mean() > 0.99, clear.mean()
    S16 = S.astype(np.float16).astype(np.float64)
    ref = M16 @ S16
    bound = N * 2.0 ** -24 * (M16 @ np.abs(S16)) + 1e-30
    assert (np.abs(Fs - ref) <= bound).all(), float((np.abs(Fs - ref) / bound).max())
    o = LG.language_features(f[idx], ws, bs, S)
    amb = o["ambiguous"]
    tol = (2.0 ** -10 + 2e-5) * o["F_abs"] + N * 2.0 ** -25 * np.abs(S).max()
    assert (np.abs(Fs - o["F"])[~amb] <= tol[~amb]).all()
    note(f"sampled {len(idx)} of {P}: ambiguous {n_amb}, resolved {int(resolved.sum())}")
